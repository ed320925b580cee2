// Zolo-eig (internal): spectral divide and conquer on the sign function.
#pragma once
#include "zcsd_internal.h"

namespace zcsd {

// batched Jacobi on blocks of at most 64 (jacobi.hip): sizes per block (device),
// A_b read (ld lda, stride sA), V_b written (n_b x n_b, ld ldv), lam_b (64 per block)
void jacobi_batched(int nblk, const int* d_sizes, const double* A, long long lda, long long sA,
                    double* V, long long ldv, long long sV, double* d_lam, hipStream_t s);

struct ZoloEigArgs {
  int n = 0;
  int batch = 1;               // independent problems of the same size
  const double* B = nullptr;  // n x n symmetric, ld ldb, problem p at B + p * sB
  long long ldb = 0, sB = 0;
  double lo = -1.0, hi = 1.0;  // spectrum bounds (every problem)
  double* V = nullptr;         // n x n eigenvectors (ld ldv, stride sV), ascending eigenvalues
  long long ldv = 0, sV = 0;
  double* lam = nullptr;       // n eigenvalues per problem (device, stride sL)
  long long sL = 0;
  int n_leaf = 64;
  double eps = 1e-15, tol = 0x1p-53;
  bool measure_offblock = true;
  bool lowp = false;           // products on the FP32 matrix cores (mixed mode)
  // keep_below < hi: only the eigenpairs below keep_below are wanted (a
  // spectral divide and conquer restricted to an interval): the first split
  // is at keep_below and the part above is finished without dividing it
  // (its columns are an orthonormal basis of that invariant subspace and its
  // eigenvalues the diagonal of the projected block, both only approximate)
  double keep_below = 1e300;
};
struct ZoloEigResult {
  int levels = 0, splits = 0, max_r = 0, failed_splits = 0;
  double max_offblock = 0.0;
  double max_coupling = 0.0;   // largest ||X||_F of the subspace-iteration step
  int full_refinements = 0;    // splits that needed the full QR step
};
ZoloEigResult zolo_eig(const ZoloEigArgs& a, Arena& ar, hipStream_t s);

// column copies described on the host: dst[:, c] for items (device descriptors)
struct CopyDesc {
  long long src_off, dst_off;  // element offsets from the base pointers
  int src_ld, dst_ld;
  int rows, cols;
};
void copy_blocks(const double* src, double* dst, const std::vector<CopyDesc>& d, Arena& ar,
                 hipStream_t s);

}  // namespace zcsd
