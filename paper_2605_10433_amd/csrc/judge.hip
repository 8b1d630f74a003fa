// Logical-failure judge: frame f fails iff it did not converge or the
// residual r = e_x xor e_hat has odd overlap with a row of the logical basis
// (a basis of ker(H_other) modulo rowspace(H)), i.e. r is not a stabilizer.
// One thread per frame; the basis rows are wave-uniform loads.  Failures
// and iteration counts are reduced per wave and added with one atomic each.
#include "internal.h"

namespace sagms {

constexpr int kJudgeBlock = 256;

__global__ void __launch_bounds__(kJudgeBlock) judge_kernel(JudgeArgs a) {
    const int64_t f = (int64_t)blockIdx.x * kJudgeBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool failed = false;
    int32_t it = 0;
    if (f < a.nframes) {
        it = a.iters[f];
        failed = a.conv[f] == 0;
        if (!failed) {
            const uint64_t* x = a.ex + f * a.wn;
            const uint64_t* e = a.ehat + f * a.wn;
            for (int t = 0; t < a.k && !failed; ++t) {
                uint32_t par = 0;
                for (int w = 0; w < a.wn; ++w) par ^= __builtin_popcountll((x[w] ^ e[w]) & a.logicals[(size_t)t * a.wn + w]);
                failed = par & 1u;
            }
        }
        if (a.fail) a.fail[f] = failed ? 1 : 0;
    }
    // wave reductions, one atomic per wave and counter
    uint64_t nfail = __builtin_popcountll(__builtin_amdgcn_ballot_w64(failed));
    uint64_t isum = (uint64_t)it;
    for (int off = 32; off > 0; off >>= 1) isum += __shfl_xor(isum, off, 64);
    if (lane == 0 && (int64_t)blockIdx.x * kJudgeBlock + threadIdx.x < a.nframes) {
        if (nfail) atomicAdd((unsigned long long*)&a.counters[0], (unsigned long long)nfail);
        if (isum) atomicAdd((unsigned long long*)&a.counters[1], (unsigned long long)isum);
    }
}

int launch_judge(const JudgeArgs& a, hipStream_t st) {
    int64_t blocks = (a.nframes + kJudgeBlock - 1) / kJudgeBlock;
    if (blocks > 0x7fffffff) return fail(SAGMS_EINVAL, "too many frames for one launch");
    hipLaunchKernelGGL(judge_kernel, dim3((unsigned)blocks), dim3(kJudgeBlock), 0, st, a);
    SAGMS_HIP(hipGetLastError());
    return SAGMS_OK;
}

}  // namespace sagms
