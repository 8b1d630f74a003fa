// Depolarizing-error sampler and syndrome kernel.
//
// Channel of Section II: qubit q of frame f is I with probability 1 - p and
// X, Y, Z with p/3 each.  The 32-bit draw of (f, q) is word q mod 4 of the
// Philox4x32-10 block (Salmon et al., SC'11) at counter
// (q / 4, f mod 2^32, f >> 32, stream) under key (seed mod 2^32, seed >> 32);
// integer thresholds T_X <= T_Y <= T_Z select X, Y, Z, so e_x = [u < T_Y] and
// e_z = [T_X <= u < T_Z].  The syndrome is s = H e_x over GF(2).
//
// A wavefront samples several frames per pass when a frame needs fewer than
// 64 Philox blocks (lanes_per_frame lanes each), so every lane evaluates one
// block.  Each lane stores its four X (and Z) bits as one 32-bit word of
// bytes in LDS; ballots over 64 consecutive qubits then give the packed
// words, which are wave-uniform.  Syndromes: for small codes every lane
// holds the packed rows of its checks in registers and takes the parity of
// (row AND e_x) with popcounts; larger codes gather the error bytes of each
// check's columns from LDS.
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
        // one 32 x 32 -> 64-bit product per multiplier (both halves at once)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// Philox pass: frames [fb, fb + 64 / lpf) (those below f_end), one block per
// lane and per stride; X / Z bits of qubit q land in byte q of the frame's
// LDS planes (padding qubits get 0).
__device__ __forceinline__ void philox_pass(const SampleArgs& a, unsigned char* xb, unsigned char* zb, int nq,
                                            int64_t fb, int64_t f_end, int lane) {
    const int fs = lane / a.lanes_per_frame;
    const int64_t f = fb + fs;
    if (f >= f_end) return;
    const uint64_t frame = a.frame0 + (uint64_t)f;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const int calls = (a.n + 3) / 4;
    for (int t = lane % a.lanes_per_frame; t < calls; t += a.lanes_per_frame) {
        uint4 u = philox4x32_10(make_uint4((uint32_t)t, (uint32_t)frame, (uint32_t)(frame >> 32), a.stream_id), k0, k1);
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
        uint32_t xw = 0, zw = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const bool in = 4 * t + b < a.n;
            xw |= (uint32_t)(in && w[b] < a.ty) << (8 * b);
            zw |= (uint32_t)(in && w[b] >= a.tx && w[b] < a.tz) << (8 * b);
        }
        *reinterpret_cast<uint32_t*>(xb + (size_t)fs * nq + 4 * t) = xw;
        *reinterpret_cast<uint32_t*>(zb + (size_t)fs * nq + 4 * t) = zw;
    }
}

// Bytes of qubits at and beyond 4 * blocks are never written by a pass:
// zero them once per wave in every frame slot of both planes.
__device__ __forceinline__ void zero_tail(const SampleArgs& a, unsigned char* xb, int nq, int lane) {
    const int fpp = 64 / a.lanes_per_frame;
    const int q0 = 4 * ((a.n + 3) / 4);
    for (int fs = 0; fs < 2 * fpp; ++fs)
        for (int q = q0 + lane; q < nq; q += 64) xb[(size_t)fs * nq + q] = 0;
}

// Small codes: n <= 64 * WN, m <= 64 * CPLS, rows of H in registers
// (JOINT: rows of 2 WN words over the (x | z) planes).
template <int WN, int CPLS, bool JOINT = false>
__global__ void __launch_bounds__(64 * kSampleWavesPerBlock) sample_kernel_rows(SampleArgs a) {
    constexpr int RW = JOINT ? 2 * WN : WN;  // words per row
    extern __shared__ unsigned char slds[];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int fpp = 64 / a.lanes_per_frame;
    constexpr int nq = 64 * WN;
    unsigned char* xb = slds + (size_t)wib * 2 * fpp * nq;
    unsigned char* zb = xb + (size_t)fpp * nq;
    const int64_t wave = (int64_t)blockIdx.x * kSampleWavesPerBlock + wib;
    const int64_t f_begin = wave * a.frames_per_wave;
    if (f_begin >= a.nframes) return;
    const int64_t f_end = min(f_begin + (int64_t)a.frames_per_wave, a.nframes);

    zero_tail(a, xb, nq, lane);
    uint64_t row[CPLS][RW];
    const int rwords = JOINT ? 2 * a.wn : a.wn;
#pragma unroll
    for (int k = 0; k < CPLS; ++k) {
        const int c = 64 * k + lane;
#pragma unroll
        for (int w = 0; w < RW; ++w) {
            const int pw = JOINT && w >= WN ? a.wn + (w - WN) : w;  // word of the row in the graph's table
            row[k][w] = (c < a.m && (w % WN) < a.wn) ? a.rows[(size_t)c * rwords + pw] : 0ull;
        }
    }

    for (int64_t fb = f_begin; fb < f_end; fb += fpp) {
        philox_pass(a, xb, zb, nq, fb, f_end, lane);
        wave_lds_sync_s();
        for (int fs = 0; fs < fpp && fb + fs < f_end; ++fs) {
            const int64_t f = fb + fs;
            uint64_t wx[WN], wzs[WN];
            uint64_t myx = 0, myz = 0, mys = 0;
#pragma unroll
            for (int w = 0; w < WN; ++w) {
                wx[w] = __builtin_amdgcn_ballot_w64(xb[(size_t)fs * nq + 64 * w + lane] != 0);
                wzs[w] = __builtin_amdgcn_ballot_w64(zb[(size_t)fs * nq + 64 * w + lane] != 0);
                if (lane == w) {
                    myx = wx[w];
                    myz = wzs[w];
                }
            }
#pragma unroll
            for (int k = 0; k < CPLS; ++k) {
                uint32_t cnt = 0;
#pragma unroll
                for (int w = 0; w < WN; ++w) cnt += __builtin_popcountll(row[k][w] & wx[w]);
                if constexpr (JOINT) {
#pragma unroll
                    for (int w = 0; w < WN; ++w) cnt += __builtin_popcountll(row[k][WN + w] & wzs[w]);
                }
                const uint64_t ws = __builtin_amdgcn_ballot_w64(cnt & 1u);
                if (lane == k) mys = ws;
            }
            if (lane < a.wn) {
                a.ex[f * a.wn + lane] = myx;
                if (a.ez) a.ez[f * a.wn + lane] = myz;
            }
            if (lane < a.wm) a.synd[f * a.wm + lane] = mys;
        }
        wave_lds_sync_s();
    }
}

// Any size: column lists of H staged in LDS (16-bit), error bytes gathered.
__global__ void __launch_bounds__(64 * kSampleWavesPerBlock) sample_kernel_gather(SampleArgs a) {
    extern __shared__ unsigned char slds[];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int fpp = 64 / a.lanes_per_frame;
    const int nq = 64 * a.wn;
    uint16_t* cols = reinterpret_cast<uint16_t*>(slds);
    const int ncols = a.m * a.dc;
    const size_t cols_bytes = ((size_t)ncols * 2 + 15) & ~(size_t)15;
    for (int t = threadIdx.x; t < ncols; t += blockDim.x) cols[t] = (uint16_t)(a.cols[t] < 0 ? 0xFFFF : a.cols[t]);
    __syncthreads();
    unsigned char* xb = slds + cols_bytes + (size_t)wib * 2 * fpp * nq;
    unsigned char* zb = xb + (size_t)fpp * nq;
    const int64_t wave = (int64_t)blockIdx.x * kSampleWavesPerBlock + wib;
    const int64_t f_begin = wave * a.frames_per_wave;
    if (f_begin >= a.nframes) return;
    const int64_t f_end = min(f_begin + (int64_t)a.frames_per_wave, a.nframes);
    zero_tail(a, xb, nq, lane);

    for (int64_t fb = f_begin; fb < f_end; fb += fpp) {
        philox_pass(a, xb, zb, nq, fb, f_end, lane);
        wave_lds_sync_s();
        for (int fs = 0; fs < fpp && fb + fs < f_end; ++fs) {
            const int64_t f = fb + fs;
            const unsigned char* x = xb + (size_t)fs * nq;
            for (int w = 0; w < a.wn; ++w) {
                const uint64_t wx = __builtin_amdgcn_ballot_w64(x[64 * w + lane] != 0);
                const uint64_t wz = __builtin_amdgcn_ballot_w64(zb[(size_t)fs * nq + 64 * w + lane] != 0);
                if (lane == 0) {
                    a.ex[f * a.wn + w] = wx;
                    if (a.ez) a.ez[f * a.wn + w] = wz;
                }
            }
            for (int k = 0; k < a.wm; ++k) {
                const int c = 64 * k + lane;
                uint32_t par = 0;
                if (c < a.m) {
                    const uint16_t* rc = cols + (size_t)c * a.dc;
                    const unsigned char* z = zb + (size_t)fs * nq;
                    for (int p = 0; p < a.dc; ++p) {
                        const uint16_t j = rc[p];  // joint graphs: n + j is byte j of the Z plane
                        if (j != 0xFFFF) par ^= j < a.n ? x[j] : z[j - a.n];
                    }
                }
                const uint64_t ws = __builtin_amdgcn_ballot_w64(par & 1u);
                if (lane == 0) a.synd[f * a.wm + k] = ws;
            }
        }
        wave_lds_sync_s();
    }
}

int launch_sample(const SampleArgs& a0, hipStream_t st) {
    SampleArgs a = a0;
    const int calls = (a.n + 3) / 4;
    int lpf = 1;
    while (lpf < calls && lpf < 64) lpf <<= 1;
    a.lanes_per_frame = lpf;
    const int fpp = 64 / lpf;
    a.frames_per_wave = fpp * a0.frames_per_wave;  // passes per wave
    int64_t waves = (a.nframes + a.frames_per_wave - 1) / a.frames_per_wave;
    int64_t blocks = (waves + kSampleWavesPerBlock - 1) / kSampleWavesPerBlock;
    if (blocks > 0x7fffffff) return fail(SAGMS_EINVAL, "too many frames for one launch");
    const dim3 grid((unsigned)blocks), block(64 * kSampleWavesPerBlock);
#define ROWS(WN, CPLS)                                                                                    \
    if (a.wn <= WN && a.wm <= CPLS) {                                                                      \
        size_t lds = (size_t)kSampleWavesPerBlock * 2 * fpp * 64 * WN;                                     \
        hipLaunchKernelGGL((sample_kernel_rows<WN, CPLS>), grid, block, lds, st, a);                      \
        SAGMS_HIP(hipGetLastError());                                                                      \
        return SAGMS_OK;                                                                                   \
    }
#define ROWS_J(WN, CPLS)                                                                                  \
    if (a.wn <= WN && a.wm <= CPLS) {                                                                      \
        size_t lds = (size_t)kSampleWavesPerBlock * 2 * fpp * 64 * WN;                                     \
        hipLaunchKernelGGL((sample_kernel_rows<WN, CPLS, true>), grid, block, lds, st, a);                \
        SAGMS_HIP(hipGetLastError());                                                                      \
        return SAGMS_OK;                                                                                   \
    }
    if (a.rows && a.joint) {
        ROWS_J(1, 1)
        ROWS_J(2, 2)
        ROWS_J(4, 4)
    } else if (a.rows) {
        ROWS(1, 1)
        ROWS(2, 1)
        ROWS(4, 2)
        ROWS(8, 4)
    }
#undef ROWS
#undef ROWS_J
    if (a.n > 0xFFFF) return fail(SAGMS_EUNSUPPORTED, "sampler supports n < 65535");
    size_t cols_bytes = ((size_t)a.m * a.dc * 2 + 15) & ~(size_t)15;
    size_t lds = cols_bytes + (size_t)kSampleWavesPerBlock * 2 * fpp * 64 * a.wn;
    if (lds > 65536) return fail(SAGMS_EUNSUPPORTED, "graph too large for the sampler's LDS");
    hipLaunchKernelGGL(sample_kernel_gather, grid, block, lds, st, a);
    SAGMS_HIP(hipGetLastError());
    return SAGMS_OK;
}

}  // namespace sagms
