// Magnification estimator of inverse ray-shooting (Thompson et al. 2009, section 1 eq. 4):
// mu_ij = N_ij / N_av, with N_av the rays a pixel receives without lensing.  One pass over the
// map: 4 bytes read and 8 bytes written per pixel, so the kernel is bound by HBM bandwidth.
#include "rs_internal.h"

namespace rs {

namespace {

// mu[b] = counts[b] / n_av for b < bins (IEEE FP64 division, correctly rounded).  Each thread
// takes four bins per step: one 16-byte load when the counts are 16-byte aligned.
__global__ void __launch_bounds__(256) k_magnification(const uint32_t *counts, int64_t bins, double n_av, double *mu)
{
    const int64_t n4 = (bins + 3) / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const bool vec_in = ((uintptr_t)counts & 15u) == 0, vec_out = ((uintptr_t)mu & 15u) == 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const int64_t b = 4 * i;
        if (b + 3 < bins && vec_in && vec_out) {
            const uint4 c = *reinterpret_cast<const uint4 *>(counts + b);
            double2 *o = reinterpret_cast<double2 *>(mu + b);
            o[0] = make_double2((double)c.x / n_av, (double)c.y / n_av);
            o[1] = make_double2((double)c.z / n_av, (double)c.w / n_av);
        } else {
            for (int j = 0; j < 4 && b + j < bins; ++j) mu[b + j] = (double)counts[b + j] / n_av;
        }
    }
}

}  // namespace

hipError_t launch_magnification(const uint32_t *counts, int64_t bins, double n_av, double *mu, hipStream_t s)
{
    const int64_t n4 = (bins + 3) / 4;
    if (n4 <= 0) return hipSuccess;
    int64_t blocks = (n4 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_magnification, dim3((unsigned)blocks), dim3(256), 0, s, counts, bins, n_av, mu);
    return hipGetLastError();
}

}  // namespace rs
