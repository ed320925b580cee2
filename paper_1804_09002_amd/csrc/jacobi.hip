// Leaf eigensolver of Zolo-eig: one workgroup per block of at most 64 x 64
// (the solve itself, cyclic Jacobi plus one refinement step, is jacobi_block).
#include <cmath>

#include "jacobi_block.h"
#include "zcsd_eig.h"
#include "zcsd_internal.h"

namespace zcsd {

__global__ __launch_bounds__(kLeafThreads) void jacobi_kernel(const int* __restrict__ sizes, const double* A,
                                                     long long lda, long long sA, double* V,
                                                     long long ldv, long long sV, double* lam) {
  __shared__ JacobiShared<kLeafMax, kLeafThreads> sh;
  const int b = blockIdx.x;
  const int n = sizes[b];
  if (n <= 0) return;
  jacobi_block(n, A + (long long)b * sA, lda, V + (long long)b * sV, ldv, lam + (long long)b * kLeafMax, sh);
}

void jacobi_batched(int nblk, const int* d_sizes, const double* A, long long lda, long long sA,
                    double* V, long long ldv, long long sV, double* d_lam, hipStream_t s) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(jacobi_kernel, dim3(nblk), dim3(kLeafThreads), 0, s, d_sizes, A, lda, sA, V, ldv, sV,
                     d_lam);
  ZCSD_CHECK_LAUNCH();
}

}  // namespace zcsd
