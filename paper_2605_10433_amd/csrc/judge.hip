// Logical-failure judge: frame f fails iff it did not converge or the
// residual r = e_x xor e_hat has odd overlap with a row of the logical basis
// (a basis of ker(H_other) modulo rowspace(H)), i.e. r is not a stabilizer.
// Joint graphs: r = (e_x | e_z) xor (x_hat | z_hat) against rows (u | v)
// whose overlap u.r_x + v.r_z is the symplectic product with a logical
// operator.
// A bounded grid of blocks strides over the frames, kJudgeUnroll frames per
// thread at a time with all their loads issued before any is used: the
// residual words stay in registers, the basis is staged in LDS (read at
// wave-uniform addresses) and every row's parity is evaluated without an
// early exit.  Failure and round counts are reduced per thread, then per
// block, and added with one atomic per block and counter.  Atomics on one
// address serialise (about 10 ns each on this GPU: 2048 of them took half of
// a 2^20-frame judge), so the grid is at most 256 blocks of 1024 threads.
#include "internal.h"

namespace sagms {

constexpr int kJudgeBlock = 1024;
constexpr int kJudgeMaxBlocks = 256;
constexpr size_t kJudgeLdsMax = 32768;

// Word w of frame f's error: the X plane, then (joint graphs) the Z plane.
__device__ __forceinline__ uint64_t error_word(const JudgeArgs& a, int64_t f, int w) {
    return w < a.wplane ? a.ex[f * a.wplane + w] : a.ez[f * a.wplane + (w - a.wplane)];
}

__device__ __forceinline__ bool judge_frame_any(const JudgeArgs& a, int64_t f) {
    const uint64_t* e = a.ehat + f * a.wn;
    uint32_t odd = 0;
    for (int t = 0; t < a.k; ++t) {
        uint32_t cnt = 0;
        for (int w = 0; w < a.wn; ++w)
            cnt += __builtin_popcountll((error_word(a, f, w) ^ e[w]) & a.logicals[(size_t)t * a.wn + w]);
        odd |= cnt;
    }
    return a.conv[f] == 0 || (odd & 1u);
}

constexpr int kJudgeUnroll = 4;

// Parity of the residual r against every basis row: 1 iff some row has odd
// overlap.
template <int WN>
__device__ __forceinline__ uint32_t judge_odd(const JudgeArgs& a, const uint64_t* lg, const uint64_t (&r)[WN]) {
    uint32_t odd = 0;
    for (int t = 0; t < a.k; ++t) {
        uint32_t cnt = 0;
#pragma unroll
        for (int w = 0; w < WN; ++w)
            if (w < a.wn) cnt += __builtin_popcountll(r[w] & lg[t * a.wn + w]);
        odd |= cnt;
    }
    return odd & 1u;
}

// WN = 0: basis and residual read from global memory (any size).
template <int WN>
__global__ void __launch_bounds__(kJudgeBlock) judge_kernel(JudgeArgs a) {
    extern __shared__ uint64_t lg[];
    __shared__ unsigned long long part[2][kJudgeBlock / 64];
    if constexpr (WN > 0) {
        for (int t = threadIdx.x; t < a.k * a.wn; t += kJudgeBlock) lg[t] = a.logicals[t];
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * kJudgeBlock;
    uint64_t nfail = 0, isum = 0;
    if constexpr (WN > 0) {
        for (int64_t f0 = (int64_t)blockIdx.x * kJudgeBlock + threadIdx.x; f0 < a.nframes;
             f0 += kJudgeUnroll * stride) {
            uint64_t r[kJudgeUnroll][WN];
            uint8_t conv[kJudgeUnroll];
            int32_t it[kJudgeUnroll];
#pragma unroll
            for (int u = 0; u < kJudgeUnroll; ++u) {
                const int64_t f = f0 + u * stride;
                const bool in = f < a.nframes;
#pragma unroll
                for (int w = 0; w < WN; ++w)
                    r[u][w] = in && w < a.wn ? error_word(a, f, w) ^ a.ehat[f * a.wn + w] : 0ull;
                conv[u] = in ? a.conv[f] : 1;
                it[u] = in ? a.iters[f] : 0;
            }
#pragma unroll
            for (int u = 0; u < kJudgeUnroll; ++u) {
                const int64_t f = f0 + u * stride;
                if (f >= a.nframes) break;
                const bool failed = conv[u] == 0 || judge_odd<WN>(a, lg, r[u]);
                if (a.fail) a.fail[f] = failed ? 1 : 0;
                nfail += failed ? 1 : 0;
                isum += (uint64_t)it[u];
            }
        }
    } else {
        for (int64_t f = (int64_t)blockIdx.x * kJudgeBlock + threadIdx.x; f < a.nframes; f += stride) {
            const bool failed = judge_frame_any(a, f);
            if (a.fail) a.fail[f] = failed ? 1 : 0;
            nfail += failed ? 1 : 0;
            isum += (uint64_t)a.iters[f];
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        nfail += __shfl_xor(nfail, off, 64);
        isum += __shfl_xor(isum, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        part[0][wid] = nfail;
        part[1][wid] = isum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s0 = 0, s1 = 0;
        for (int t = 0; t < kJudgeBlock / 64; ++t) {
            s0 += part[0][t];
            s1 += part[1][t];
        }
        if (s0) atomicAdd((unsigned long long*)&a.counters[0], s0);
        if (s1) atomicAdd((unsigned long long*)&a.counters[1], s1);
    }
}

int launch_judge(const JudgeArgs& a, hipStream_t st) {
    int64_t blocks = (a.nframes + kJudgeBlock - 1) / kJudgeBlock;
    if (blocks > kJudgeMaxBlocks) blocks = kJudgeMaxBlocks;
    const size_t lds = (size_t)a.k * a.wn * sizeof(uint64_t);
    const dim3 grid((unsigned)blocks), block(kJudgeBlock);
#define WNS(WN)                                                                      \
    if (lds <= kJudgeLdsMax && a.wn <= WN) {                                         \
        hipLaunchKernelGGL((judge_kernel<WN>), grid, block, lds, st, a);             \
        SAGMS_HIP(hipGetLastError());                                                \
        return SAGMS_OK;                                                             \
    }
    WNS(1)
    WNS(2)
    WNS(4)
    WNS(8)
    WNS(16)
#undef WNS
    hipLaunchKernelGGL((judge_kernel<0>), grid, block, 0, st, a);
    SAGMS_HIP(hipGetLastError());
    return SAGMS_OK;
}

}  // namespace sagms
