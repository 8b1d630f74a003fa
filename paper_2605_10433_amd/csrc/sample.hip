// Depolarizing-error sampler and syndrome kernel.
//
// Channel of Section II: qubit q of frame f is I with probability 1 - p and
// X, Y, Z with p/3 each.  The 32-bit draw of (f, q) is word q mod 4 of the
// Philox4x32-10 block (Salmon et al., SC'11) at counter
// (q / 4, f mod 2^32, f >> 32, stream) under key (seed mod 2^32, seed >> 32);
// integer thresholds T_X <= T_Y <= T_Z select X, Y, Z, so e_x = [u < T_Y] and
// e_z = [T_X <= u < T_Z].  The syndrome is s = H e_x over GF(2).
//
// One wavefront handles one frame at a time: lanes evaluate Philox blocks,
// write the X / Z bit of every qubit to LDS as bytes, then ballots over
// 64 consecutive qubits (or checks) produce the packed words.
#include "internal.h"

namespace sagms {

constexpr int kSampleWavesPerBlock = 4;

__device__ __forceinline__ void wave_lds_sync_s() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Philox4x32-10 block function (Salmon et al., SC'11, the Philox S-box with
// 10 rounds, multipliers 0xD2511F53 / 0xCD9E8D57, key schedule by the Weyl
// increments 0x9E3779B9 / 0xBB67AE85).
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

__global__ void __launch_bounds__(64 * kSampleWavesPerBlock) sample_kernel(SampleArgs a) {
    extern __shared__ unsigned char slds[];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int nq = (a.n + 63) & ~63;            // qubit bytes per plane, padded to 64
    unsigned char* xb = slds + (size_t)wib * 2 * nq;
    unsigned char* zb = xb + nq;
    const int64_t wave = (int64_t)blockIdx.x * kSampleWavesPerBlock + wib;
    const int64_t f_begin = wave * a.frames_per_wave;
    if (f_begin >= a.nframes) return;
    const int64_t f_end = min(f_begin + (int64_t)a.frames_per_wave, a.nframes);
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const int calls = (a.n + 3) / 4;
    for (int q = a.n + lane; q < nq; q += 64) {  // padding qubits stay zero
        xb[q] = 0;
        zb[q] = 0;
    }

    for (int64_t f = f_begin; f < f_end; ++f) {
        const uint64_t frame = a.frame0 + (uint64_t)f;
        for (int t = lane; t < calls; t += 64) {
            uint4 u = philox4x32_10(make_uint4((uint32_t)t, (uint32_t)frame, (uint32_t)(frame >> 32), a.stream_id),
                                    k0, k1);
            const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                int q = 4 * t + b;
                if (q < a.n) {
                    xb[q] = w[b] < a.ty;
                    zb[q] = (w[b] >= a.tx) & (w[b] < a.tz);
                }
            }
        }
        wave_lds_sync_s();
        for (int wd = 0; wd < a.wn; ++wd) {
            const int q = 64 * wd + lane;
            uint64_t wx = __builtin_amdgcn_ballot_w64(xb[q] != 0);
            uint64_t wz = __builtin_amdgcn_ballot_w64(zb[q] != 0);
            if (lane == 0) {
                a.ex[f * a.wn + wd] = wx;
                if (a.ez) a.ez[f * a.wn + wd] = wz;
            }
        }
        for (int wd = 0; wd < a.wm; ++wd) {
            const int c = 64 * wd + lane;
            uint32_t par = 0;
            if (c < a.m) {
                const int32_t* row = a.cols + (size_t)c * a.dc;
                for (int p = 0; p < a.dc; ++p) {
                    int j = row[p];
                    if (j >= 0) par ^= xb[j];
                }
            }
            uint64_t ws = __builtin_amdgcn_ballot_w64(par & 1u);
            if (lane == 0) a.synd[f * a.wm + wd] = ws;
        }
        wave_lds_sync_s();
    }
}

int launch_sample(const SampleArgs& a, hipStream_t st) {
    int64_t waves = (a.nframes + a.frames_per_wave - 1) / a.frames_per_wave;
    int64_t blocks = (waves + kSampleWavesPerBlock - 1) / kSampleWavesPerBlock;
    if (blocks > 0x7fffffff) return fail(SAGMS_EINVAL, "too many frames for one launch");
    const int nq = (a.n + 63) & ~63;
    size_t lds = (size_t)kSampleWavesPerBlock * 2 * nq;
    hipLaunchKernelGGL(sample_kernel, dim3((unsigned)blocks), dim3(64 * kSampleWavesPerBlock), lds, st, a);
    SAGMS_HIP(hipGetLastError());
    return SAGMS_OK;
}

}  // namespace sagms
