// Device self-test of the generator's short arithmetic: for every uniform
// u = (2k + 1) 2^-24, k < 2^23, the logarithm computed with div_gen must
// equal the one computed with the compiler's IEEE division, the kernels'
// rearranged -2 ln u and quarter-turn sine and cosine (from u 2^32) must
// equal -2 times that logarithm and the plain sincos_turn(u), and sqrt_gen of
// -2 ln u must equal the IEEE square root, bit for bit.  One thread per k;
// mismatches are counted with vector atomics.
#include "kernels.h"

namespace procmv {

namespace {

__global__ __launch_bounds__(256) void selftest_generator_kernel(unsigned* count)
{
    const uint32_t k = blockIdx.x * 256u + threadIdx.x;
    if (k >= (1u << 23)) return;
    const float u = (float)(k * 2u + 1u) * 5.9604644775390625e-8f;
    const float l = ln_unit<false>(u);
    const float l_ieee = ln_unit<true>(u);
    const float a = -2.0f * l_ieee;
    // any word x with x >> 9 == k draws this u; take the extremes
    const float z_lo = unit_2p32(k << 9), z_hi = unit_2p32((k << 9) | 0x1FFu);
    float s_ref, c_ref, s_k, c_k;
    sincos_turn(u, s_ref, c_ref);
    sincos_2p32(z_lo, s_k, c_k);
    bool bad_ln = __float_as_uint(l) != __float_as_uint(l_ieee);
    bad_ln |= __float_as_uint(neg2_ln_2p32(z_lo)) != __float_as_uint(a);
    bad_ln |= __float_as_uint(z_hi) != __float_as_uint(z_lo);
    bad_ln |= __float_as_uint(s_k) != __float_as_uint(s_ref);
    bad_ln |= __float_as_uint(c_k) != __float_as_uint(c_ref);
    const bool bad_sqrt = __float_as_uint(sqrt_gen(a)) != __float_as_uint(__builtin_sqrtf(a));
    if (bad_ln) atomicAdd(&count[0], 1u);
    if (bad_sqrt) atomicAdd(&count[1], 1u);
}

__global__ void zero2_kernel(unsigned* count)
{
    if (threadIdx.x < 2) count[threadIdx.x] = 0u;
}

}  // namespace

hipError_t launch_selftest_generator(unsigned* count, hipStream_t s)
{
    hipLaunchKernelGGL(zero2_kernel, dim3(1), dim3(64), 0, s, count);
    hipLaunchKernelGGL(selftest_generator_kernel, dim3((1u << 23) / 256), dim3(256), 0, s, count);
    return hipGetLastError();
}

}  // namespace procmv
