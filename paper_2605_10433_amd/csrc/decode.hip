// Decode kernels: MS / SMS / SAGMS (one kernel, gain table) and BP.
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
//     VN     every variable sums L0 and its incoming c2v messages in
//            ascending check order and stores the posterior (eq. (bp4_vn)).
//   The hard decision is e_hat_j = [posterior_j < 0].
// Posteriors and v2c messages are never -0.0 (L0 is read as L0 + 0.0f and
// every later value is a sum or a difference of finite floats starting from
// it), so sign bits and "< 0" agree and the kernel uses sign bits.
#include "internal.h"

namespace sagms {

constexpr uint32_t kSign = 0x80000000u;
constexpr int kWavesPerBlock = 4;

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

template <int DC, int DV, int CPL, int VPL, bool BP>
__global__ void __launch_bounds__(64 * kWavesPerBlock) decode_kernel(DecodeArgs a) {
    extern __shared__ float lds_all[];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    float* lds = lds_all + wib * a.L.words;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    const int64_t f_begin = wave * a.frames_per_wave;
    if (f_begin >= a.nframes) return;
    const int64_t f_end = min(f_begin + (int64_t)a.frames_per_wave, a.nframes);
    const int cw = a.L.cw;

    // graph tables and priors: loaded once per wave
    uint32_t caddr[CPL][DC];
    uint32_t vaddr[VPL][DV];
#pragma unroll
    for (int k = 0; k < CPL; ++k)
#pragma unroll
        for (int p = 0; p < DC; ++p) caddr[k][p] = a.cn_addr[(k * DC + p) * 64 + lane];
#pragma unroll
    for (int k = 0; k < VPL; ++k)
#pragma unroll
        for (int r = 0; r < DV; ++r) vaddr[k][r] = a.vn_addr[(k * DV + r) * 64 + lane];
    float L0[VPL];
#pragma unroll
    for (int k = 0; k < VPL; ++k) {
        int j = k * 64 + lane;
        L0[k] = j < a.n ? a.llr0[j] + 0.0f : __builtin_inff();
    }
    bool cvalid[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) cvalid[k] = k * 64 + lane < a.m;
    for (int t = lane; t < 2 * (cw + 1); t += 64) lds[a.L.gain0 + t] = a.gains[t];
    if (lane == 0) {
        lds[a.L.zero] = 0.0f;
        lds[a.L.padpost] = __builtin_inff();
    }

    for (int64_t f = f_begin; f < f_end; ++f) {
        uint32_t sb[CPL];  // original syndrome bit of each owned check, at the sign position
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            uint64_t word = k < a.wm ? a.synd[f * a.wm + k] : 0ull;
            sb[k] = cvalid[k] ? (uint32_t)((word >> lane) & 1ull) << 31 : 0u;
        }
        float post[VPL];
#pragma unroll
        for (int k = 0; k < VPL; ++k) {
            post[k] = L0[k];
            lds[a.L.post0 + k * 64 + lane] = L0[k];
        }
        float c2v[CPL][DC];
#pragma unroll
        for (int k = 0; k < CPL; ++k)
#pragma unroll
            for (int p = 0; p < DC; ++p) c2v[k][p] = 0.0f;
        wave_lds_sync();

        int it = 0;
        bool conv = false;
        while (true) {
            // top of the round: v2c, hard-decision parity, residual syndrome
            float v[CPL][DC];
            bool unsat[CPL];
            int w = 0;
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                uint32_t hd = 0;
#pragma unroll
                for (int p = 0; p < DC; ++p) {
                    float pj = lds[caddr[k][p]];
                    v[k][p] = pj - c2v[k][p];
                    hd ^= __float_as_uint(pj);
                }
                unsat[k] = cvalid[k] && ((hd ^ sb[k]) & kSign);
                w += __builtin_popcountll(ballot(unsat[k]));
            }
            if (w == 0) {
                conv = true;
                break;
            }
            if (it == a.lmax) break;
            ++it;
            // CN update
            const float2 gg = *reinterpret_cast<const float2*>(&lds[a.L.gain0 + 2 * w]);
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                uint32_t par = sb[k];
#pragma unroll
                for (int p = 0; p < DC; ++p) par ^= __float_as_uint(v[k][p]);
                par &= kSign;
                if constexpr (BP) {
                    float mag[DC];
                    bp_magnitudes<DC>(v[k], mag);
#pragma unroll
                    for (int p = 0; p < DC; ++p)
                        c2v[k][p] = __uint_as_float(__float_as_uint(mag[p]) |
                                                    ((__float_as_uint(v[k][p]) ^ par) & kSign));
                } else {
                    const float alpha = unsat[k] ? gg.y : gg.x;
                    float m1 = __builtin_inff(), m2 = __builtin_inff();
#pragma unroll
                    for (int p = 0; p < DC; ++p) {
                        float x = fabsf(v[k][p]);
                        m2 = __builtin_amdgcn_fmed3f(m1, x, m2);
                        m1 = fminf(m1, x);
                    }
                    const float s1 = alpha * m1, s2 = alpha * m2;
#pragma unroll
                    for (int p = 0; p < DC; ++p) {
                        float mag = fabsf(v[k][p]) == m1 ? s2 : s1;
                        c2v[k][p] = __uint_as_float(__float_as_uint(mag) |
                                                    ((__float_as_uint(v[k][p]) ^ par) & kSign));
                    }
                }
#pragma unroll
                for (int p = 0; p < DC; ++p) lds[p * cw + k * 64 + lane] = c2v[k][p];
            }
            wave_lds_sync();
            // VN update: posterior in ascending check order
#pragma unroll
            for (int k = 0; k < VPL; ++k) {
                float s = L0[k];
#pragma unroll
                for (int r = 0; r < DV; ++r) s = s + lds[vaddr[k][r]];
                post[k] = s;
                lds[a.L.post0 + k * 64 + lane] = s;
            }
            wave_lds_sync();
        }

        // outputs: hard decisions, round count, convergence flag
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
}

// Waves per block: up to kWavesPerBlock, as many as fit in 64 KiB of LDS.
static int waves_per_block(const DecodeLayout& L) {
    int w = (int)(65536 / ((size_t)L.words * sizeof(float)));
    return w < 1 ? 1 : (w > kWavesPerBlock ? kWavesPerBlock : w);
}

template <int DC, int DV, int CPL, int VPL>
static int launch_shape(bool bp, const DecodeArgs& a, hipStream_t st) {
    if ((size_t)a.L.words * sizeof(float) > 65536) return fail(SAGMS_EUNSUPPORTED, "graph too large for one wave's LDS");
    const int wpb = waves_per_block(a.L);
    int64_t waves = (a.nframes + a.frames_per_wave - 1) / a.frames_per_wave;
    int64_t blocks = (waves + wpb - 1) / wpb;
    if (blocks > 0x7fffffff) return fail(SAGMS_EINVAL, "too many frames for one launch");
    size_t lds = (size_t)wpb * a.L.words * sizeof(float);
    if (bp)
        hipLaunchKernelGGL((decode_kernel<DC, DV, CPL, VPL, true>), dim3((unsigned)blocks), dim3(64 * wpb), lds, st, a);
    else
        hipLaunchKernelGGL((decode_kernel<DC, DV, CPL, VPL, false>), dim3((unsigned)blocks), dim3(64 * wpb), lds, st,
                           a);
    SAGMS_HIP(hipGetLastError());
    return SAGMS_OK;
}

int launch_decode(const DecodeShape& s, bool bp, const DecodeArgs& a, int, hipStream_t st) {
#define SHAPE(DC, DV, CPL, VPL) \
    if (s.dc == DC && s.dv == DV && s.cpl == CPL && s.vpl == VPL) return launch_shape<DC, DV, CPL, VPL>(bp, a, st);
    SHAPE(4, 2, 1, 1)
    SHAPE(6, 3, 1, 1)
    SHAPE(10, 5, 1, 2)
    SHAPE(16, 8, 1, 2)
    SHAPE(10, 5, 2, 4)
    SHAPE(16, 8, 2, 4)
    SHAPE(6, 3, 4, 8)
    SHAPE(8, 4, 4, 8)
    SHAPE(10, 5, 8, 16)
#undef SHAPE
    return fail(SAGMS_EUNSUPPORTED, "no decode kernel for shape dc=%d dv=%d cpl=%d vpl=%d", s.dc, s.dv, s.cpl, s.vpl);
}

}  // namespace sagms
