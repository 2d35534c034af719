// Device helpers of the pixel-level smoothers shared by their kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace mlcr {

// In-place Cholesky (lower, row-major kk x kk in LDS) by one workgroup; a
// non-positive pivot is replaced by 1 and reported (returns false).
__device__ inline bool lds_cholesky(double *a, int kk, double *flag) {
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) *flag = 0.0;
    __syncthreads();
    for (int j = 0; j < kk; j++) {
        if (tid == 0) {
            const double piv = a[j * kk + j];
            if (!(piv > 0.0)) *flag = 1.0;
            a[j * kk + j] = piv > 0.0 ? sqrt(piv) : 1.0;
        }
        __syncthreads();
        const double djj = a[j * kk + j];
        for (int i = j + 1 + tid; i < kk; i += nt) a[i * kk + j] /= djj;
        __syncthreads();
        const int rem = kk - j - 1;
        for (int e = tid; e < rem * rem; e += nt) {
            const int i = j + 1 + e / rem, c = j + 1 + e % rem;
            if (c <= i) a[i * kk + c] -= a[i * kk + j] * a[c * kk + j];
        }
        __syncthreads();
    }
    return *flag == 0.0;
}

}  // namespace mlcr
