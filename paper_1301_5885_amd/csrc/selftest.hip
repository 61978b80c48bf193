// Device arithmetic exposed for tests: the FP64 exponential of the pair
// kernels (e^{-kappa rho} in K1..K4, Section 2.1 eq. (Eq_Ls)).
#include "gabi_internal.h"
#include "pair_math.h"

namespace gabi {

__global__ __launch_bounds__(kBlock) void exp_neg_kernel(const double *__restrict__ t, int64_t n,
                                                         double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = exp_neg_f64(t[i]);
}

}  // namespace gabi

extern "C" int gabi_selftest_exp_neg(int device, int64_t n, const double *t, double *out) {
    if (n < 1 || n > (int64_t(1) << 28) || !t || !out) return GABI_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!(t[i] >= 0.0) || !std::isfinite(t[i])) return GABI_EINVAL;
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        return GABI_EDEVICE;
    }
    double *d = nullptr;
    if (hipMalloc(&d, sizeof(double) * 2 * (size_t)n) != hipSuccess) {
        (void)hipGetLastError();
        return GABI_ENOMEM;
    }
    hipError_t e = hipMemcpy(d, t, sizeof(double) * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(gabi::exp_neg_kernel, dim3((unsigned)((n + gabi::kBlock - 1) / gabi::kBlock)),
                           dim3(gabi::kBlock), 0, 0, d, n, d + n);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpy(out, d + n, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return GABI_EDEVICE;
    }
    return GABI_OK;
}
