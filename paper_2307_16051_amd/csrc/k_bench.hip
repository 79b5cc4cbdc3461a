// k_bench.hip -- measurement helper, not a step of the method: the rate the
// matrix cores reach on this device, which the factorisation's roofline is
// also set against (next to the published dense peak).
#include "n3p_internal.hpp"

namespace n3p {

template <typename T> struct mfma_rate_op;
template <> struct mfma_rate_op<f16> {
    typedef h8 vec;
    static __device__ __forceinline__ f32x16 op(vec a, vec b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct mfma_rate_op<bf16> {
    typedef b8 vec;
    static __device__ __forceinline__ f32x16 op(vec a, vec b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

// Every wavefront keeps NACC independent 32x32 FP32 accumulators and issues
// v_mfma_f32_32x32x16 back to back `iters` times on each, with register
// operands.  With every operand entry 1/32, one instruction adds
// 16 / 1024 = 1/64 to each accumulator entry, so the sum of a lane's 16 * NACC
// entries is 2 * iters exactly (FP32, iters <= 2^20); each lane stores it, so
// none of the work is dead code and the result checks that it was done.
constexpr int RATE_NACC = 8;

template <typename T>
__global__ __launch_bounds__(256) void k_mfma_rate(int iters, float *__restrict__ out)
{
    typedef typename mfma_rate_op<T>::vec vec;
    vec a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = (T)(1.0f / 32.0f);
        b[e] = (T)(1.0f / 32.0f);
    }
    f32x16 acc[RATE_NACC];
#pragma unroll
    for (int q = 0; q < RATE_NACC; ++q)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[q][e] = 0.0f;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int q = 0; q < RATE_NACC; ++q) acc[q] = mfma_rate_op<T>::op(a, b, acc[q]);
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < RATE_NACC; ++q)
#pragma unroll
        for (int e = 0; e < 16; ++e) s += acc[q][e];
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

hipError_t launch_mfma_rate(int prec, int blocks, int iters, float *out, double *flops,
                            hipStream_t s)
{
    if (blocks < 1 || iters < 1 || iters > (1 << 20)) return hipErrorInvalidValue;
    switch (prec) {
    case N3P_FP16: hipLaunchKernelGGL(k_mfma_rate<f16>, dim3(blocks), dim3(256), 0, s, iters, out); break;
    case N3P_BF16: hipLaunchKernelGGL(k_mfma_rate<bf16>, dim3(blocks), dim3(256), 0, s, iters, out); break;
    default: return hipErrorInvalidValue;
    }
    // 4 wavefronts per workgroup, RATE_NACC instructions of 2*32*32*16 flop per step
    *flops = (double)blocks * 4.0 * (double)iters * RATE_NACC * 2.0 * 32 * 32 * 16;
    return hipGetLastError();
}

}  // namespace n3p
