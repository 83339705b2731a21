// Test helper (not part of the product): compares the library's recip() with the IEEE
// division 1.0f / z for all 2^32 bit patterns on the GPU.
#include <hip/hip_runtime.h>

#include "kf_device.h"

namespace {

__global__ __launch_bounds__(256) void recip_check_kernel(uint32_t chunk, unsigned long long* bad)
{
    const uint32_t bits = (chunk << 26) | (blockIdx.x * 256u + threadIdx.x);
    const float z = __builtin_bit_cast(float, bits);
    const float fast = kf::recip(z), ieee = 1.0f / z;
    if (__builtin_bit_cast(uint32_t, fast) != __builtin_bit_cast(uint32_t, ieee)) atomicAdd(bad, 1ull);
}

}  // namespace

// Number of 32-bit inputs for which recip(z) and 1.0f / z differ in any bit; -1 on a HIP error.
extern "C" long long kf_test_recip_mismatches(void)
{
    unsigned long long* bad = nullptr;
    if (hipMalloc(&bad, sizeof *bad) != hipSuccess) return -1;
    unsigned long long host = 0;
    bool ok = hipMemcpy(bad, &host, sizeof host, hipMemcpyHostToDevice) == hipSuccess;
    for (uint32_t chunk = 0; ok && chunk < 64; ++chunk) {
        hipLaunchKernelGGL(recip_check_kernel, dim3(1u << 18), dim3(256), 0, 0, chunk, bad);
        ok = hipGetLastError() == hipSuccess;
    }
    ok = ok && hipMemcpy(&host, bad, sizeof host, hipMemcpyDeviceToHost) == hipSuccess;
    ok = (hipFree(bad) == hipSuccess) && ok;
    return ok ? (long long)host : -1;
}
