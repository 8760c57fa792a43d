// Exhaustive device check of the shortened arithmetic in device_math.hpp:
// the quotient and square-root sequences that Box-Muller uses must equal the
// correctly rounded IEEE operations on every argument they can receive.
//
//   div_log_quotient(m - 1, m + 1) == (m - 1) / (m + 1)  for every float m
//                                     in [0.70, 1.42]
//   sqrt_radius(x) == sqrt(x)       for x = 0 and every float x in
//                                     [2^-96, 64]
//
// Built for gfx950 with the library's flags (correctly rounded `/` and
// sqrt), so the right-hand sides are the IEEE operations.  Test code only.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../paper_2606_14603_amd/csrc/device_math.hpp"

namespace {

// mismatches and the smallest mismatching argument's bits
struct Result {
    unsigned long long bad;
    uint32_t first;
    uint32_t pad;
};

__global__ void k_div(uint32_t lo, uint32_t n, Result* res)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t bits = lo + i;
    const float m = __uint_as_float(bits);
    const float a = m - 1.0f, b = m + 1.0f;
    const float fast = mabm::div_log_quotient(a, b);
    const float ieee = a / b;
    if (__float_as_uint(fast) != __float_as_uint(ieee)) {
        atomicAdd(&res->bad, 1ull);
        atomicMin(&res->first, bits);
    }
}

__global__ void k_sqrt(uint32_t lo, uint32_t n, Result* res)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t bits = lo + i;
    const float x = __uint_as_float(bits);
    const float fast = mabm::sqrt_radius(x);
    const float ieee = __builtin_sqrtf(x);
    if (__float_as_uint(fast) != __float_as_uint(ieee)) {
        atomicAdd(&res->bad, 1ull);
        atomicMin(&res->first, bits);
    }
}

int run(void (*kernel)(uint32_t, uint32_t, Result*), uint32_t lo, uint32_t hi,
        unsigned long long* bad, uint32_t* first)
{
    Result* d = nullptr;
    if (hipMalloc(&d, sizeof(Result)) != hipSuccess) return -1;
    const Result init{0ull, 0xFFFFFFFFu, 0u};
    int rc = 0;
    if (hipMemcpy(d, &init, sizeof(Result), hipMemcpyHostToDevice) != hipSuccess) rc = -2;
    const uint32_t n = hi - lo + 1u;
    const uint32_t block = 256;
    if (rc == 0) {
        hipLaunchKernelGGL(kernel, dim3((n + block - 1) / block), dim3(block), 0, 0, lo, n, d);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) rc = -3;
    }
    Result out{};
    if (rc == 0 && hipMemcpy(&out, d, sizeof(Result), hipMemcpyDeviceToHost) != hipSuccess)
        rc = -4;
    hipFree(d);
    *bad = out.bad;
    *first = out.first;
    return rc;
}

}  // namespace

// Checks the bit range [lo, hi] of float arguments; returns 0 on success
// (then *bad holds the mismatch count and *first the smallest mismatching
// argument's bits, 0xFFFFFFFF if none), < 0 on a HIP error.
extern "C" int math_check_div(uint32_t lo, uint32_t hi, unsigned long long* bad, uint32_t* first)
{
    if (hi < lo) return -5;
    return run(k_div, lo, hi, bad, first);
}

extern "C" int math_check_sqrt(uint32_t lo, uint32_t hi, unsigned long long* bad,
                               uint32_t* first)
{
    if (hi < lo) return -5;
    return run(k_sqrt, lo, hi, bad, first);
}
