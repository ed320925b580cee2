// FP64 refinement of an approximate symmetric eigendecomposition (used by the
// mixed-precision mode, whose Zolo-eig runs its products on the FP32 matrix
// cores).
//
// Iteration (Ogita and Aishima, "Iterative refinement for symmetric eigenvalue
// decomposition", Japan J. Indust. Appl. Math. 35, 2018): for X ~ V,
//   R = I - X^T X,  S = X^T B X,  lt_i = S_ii / (1 - R_ii),
//   delta = 2 (||S - diag(lt)||_2 + ||B||_2 ||R||_2),
//   E_ij = (S_ij + lt_j R_ij) / (lt_j - lt_i)  if |lt_i - lt_j| > delta,
//   E_ij = R_ij / 2                            otherwise,
//   X <- X + X E,
// which converges quadratically for the eigenvectors of well-separated
// eigenvalues and keeps X orthonormal to working accuracy.  The 2-norms are
// power-iteration estimates (doubled), ||B||_2 comes from the spectral
// interval, and a pair takes the first-order correction only while it is
// small (|lt_j - lt_i| > 64 |S_ij + lt_j R_ij|).  Eigenvalues
// still closer than delta after the last iteration form clusters whose
// invariant subspace is accurate but whose basis is not an eigenbasis; each
// cluster's block X_c^T B X_c is diagonalised in FP64 (Jacobi up to 64, Zolo-eig
// above) and X_c rotated.  Columns end sorted by ascending eigenvalue.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <vector>

#include "zcsd_api_guard.h"
#include "zcsd_eig.h"
#include "zcsd_internal.h"

namespace zcsd {

// lt_i = S_ii / G_ii (G = X^T X, so 1 - R_ii = G_ii)
__global__ void oa_lambda_kernel(int n, const double* __restrict__ S, const double* __restrict__ G,
                                 double* lt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) lt[i] = S[i + (long long)i * n] / G[i + (long long)i * n];
}

// E (in place over S) from S, G = X^T X and lt; delta decides the clustered pairs;
// also D (over G) = S - diag(lt) is not needed afterwards
__global__ void oa_correction_kernel(int n, double* S, const double* __restrict__ G,
                                     const double* __restrict__ lt, double delta) {
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    const double r = ((i == j) ? 1.0 : 0.0) - G[e];
    const double d = lt[j] - lt[i];
    const double num = S[e] + lt[j] * r;
    // separated pairs take the first-order correction while it is small;
    // the others are only re-orthogonalised this step
    S[e] = (i != j && fabs(d) > delta && fabs(d) > 64.0 * fabs(num)) ? num / d : 0.5 * r;
  }
}

// M = S - diag(lt) (into Ms) and Rm = I - G
__global__ void oa_residuals_kernel(int n, const double* __restrict__ S, const double* __restrict__ G,
                                    const double* __restrict__ lt, double* Ms, double* Rm) {
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    Ms[e] = S[e] - ((i == j) ? lt[i] : 0.0);
    Rm[e] = ((i == j) ? 1.0 : 0.0) - G[e];
  }
}

// x = y / sqrt(ss[0]) (ss[0] = ||y||^2; x = y when it is zero)
__global__ void normalize_kernel(int n, const double* __restrict__ y, const double* __restrict__ ss,
                                 double* x) {
  const double nr = sqrt(ss[0]);
  const double f = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    x[i] = y[i] * f;
}

// x_i *= 1 + (hash(i) in [-1/2, 1/2)): a start that is not orthogonal to any
// particular singular vector
__global__ void perturb_kernel(int n, double* x) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    unsigned long long z = (unsigned long long)i * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL;
    z = (z ^ (z >> 31)) * 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 29;
    x[i] *= 1.0 + ((double)(z >> 11) * 0x1p-53 - 0.5);
  }
}

__global__ void fill_kernel(int n, double v, double* x) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = v;
}

// ||M||_2 of a symmetric n x n matrix by power iteration (device, one readback);
// the estimate is from below, so the caller adds a safety factor
static double power_norm2(int n, const double* M, int iters, Arena& ar, hipStream_t s) {
  ArenaScope sc(ar);
  double* x = ar.dalloc(n);
  double* y = ar.dalloc(n);
  double* ss = ar.dalloc(1);
  const unsigned g = (unsigned)std::max(1, std::min((n + 255) / 256, 1024));
  hipLaunchKernelGGL(fill_kernel, dim3(g), dim3(256), 0, s, n, 1.0 / std::sqrt((double)n), x);
  ZCSD_CHECK_LAUNCH();
  hipLaunchKernelGGL(perturb_kernel, dim3(g), dim3(256), 0, s, n, x);
  ZCSD_CHECK_LAUNCH();
  for (int it = 0; it < iters; ++it) {
    GemmBatch m;
    m.m = n; m.n = 1; m.k = n;
    m.A = M; m.lda = n; m.B = x; m.ldb = n; m.C = y; m.ldc = n;
    dgemm(m, s);
    sumsq(1, n, 1, y, n, 0, ss, ar, s);
    hipLaunchKernelGGL(normalize_kernel, dim3(g), dim3(256), 0, s, n, y, ss, x);
    ZCSD_CHECK_LAUNCH();
  }
  double h = 0.0;
  d2h(&h, ss, sizeof(double), s);
  return std::sqrt(h);
}

EigRefineResult eig_refine(int n, const double* B, long long ldb, double* X, double* lam,
                           double bnorm2, int iters, Arena& ar, hipStream_t s) {
  EigRefineResult res;
  const long long nn = (long long)n * n;
  ArenaScope scope(ar);
  double* G = ar.dalloc(nn);
  double* T = ar.dalloc(nn);
  double* S = ar.dalloc(nn);
  double* Xn = ar.dalloc(nn);
  double* lt = ar.dalloc(n);
  const unsigned gx = (unsigned)std::max<long long>(1, std::min<long long>((nn + 255) / 256, 4096));
  double delta = 0.0;
  auto products = [&]() {
    GemmBatch g;
    g.transA = 1;
    g.m = n; g.n = n; g.k = n;
    g.A = X; g.lda = n; g.B = X; g.ldb = n; g.C = G; g.ldc = n;
    dgemm(g, s);  // G = X^T X
    GemmBatch t;
    t.m = n; t.n = n; t.k = n;
    t.A = B; t.lda = ldb; t.B = X; t.ldb = n; t.C = T; t.ldc = n;
    dgemm(t, s);  // T = B X
    GemmBatch u;
    u.transA = 1;
    u.m = n; u.n = n; u.k = n;
    u.A = X; u.lda = n; u.B = T; u.ldb = n; u.C = S; u.ldc = n;
    dgemm(u, s);  // S = X^T B X
    hipLaunchKernelGGL(oa_lambda_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, S, G, lt);
    ZCSD_CHECK_LAUNCH();
    // 2-norms of S - diag(lt) and I - X^T X by power iteration (a lower
    // estimate; doubled), into the buffers T and Xn that are free here
    hipLaunchKernelGGL(oa_residuals_kernel, dim3(gx), dim3(256), 0, s, n, S, G, lt, T, Xn);
    ZCSD_CHECK_LAUNCH();
    const double a = 2.0 * power_norm2(n, T, 20, ar, s);
    const double b = 2.0 * power_norm2(n, Xn, 20, ar, s);
    delta = 2.0 * (a + std::sqrt(bnorm2) * b);
    return a;
  };
  // iterate until the off-diagonal part of S is at the rounding level of the
  // products (a few sqrt(n) u ||B|| in the 2-norm), at most `iters` corrections
  const double floor_off = 16.0 * 0x1p-53 * std::sqrt((double)n) * std::sqrt(bnorm2);
  res.offdiag = products();
  res.delta = delta;
  if (log_enabled())
    std::fprintf(stderr, "[zcsd] refine start: ||S - diag||_2 ~ %.3e, delta %.3e\n", res.offdiag, delta);
  while (res.iters < iters && res.offdiag > floor_off) {
    hipLaunchKernelGGL(oa_correction_kernel, dim3(gx), dim3(256), 0, s, n, S, G, lt, delta);
    ZCSD_CHECK_LAUNCH();
    copy_scale(1, n, n, 1.0, X, n, 0, Xn, n, 0, s);
    GemmBatch g;
    g.m = n; g.n = n; g.k = n;
    g.A = X; g.lda = n; g.B = S; g.ldb = n; g.C = Xn; g.ldc = n;
    g.beta = 1.0;
    dgemm(g, s);  // Xn = X + X E
    copy_scale(1, n, n, 1.0, Xn, n, 0, X, n, 0, s);
    ++res.iters;
    res.offdiag = products();
    res.delta = delta;
    if (log_enabled())
      std::fprintf(stderr, "[zcsd] refine step %d: ||S - diag||_2 ~ %.3e, delta %.3e\n", res.iters,
                   res.offdiag, delta);
  }
  std::vector<double> lh(n);
  d2h(lh.data(), lt, n * sizeof(double), s);
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return lh[x] < lh[y]; });
  std::vector<std::vector<int>> clusters;
  for (int a = 0; a < n;) {
    int b = a + 1;
    while (b < n && lh[ord[b]] - lh[ord[b - 1]] <= delta) ++b;
    if (b - a > 1) clusters.emplace_back(ord.begin() + a, ord.begin() + b);
    a = b;
  }
  res.converged = res.offdiag <= floor_off;
  res.clusters = (int)clusters.size();
  for (const auto& c : clusters) {
    const int m = (int)c.size();
    res.max_cluster = std::max(res.max_cluster, m);
    ArenaScope cs(ar);
    // Xc = X(:, c), Sc = Xc^T B Xc
    double* Sc = ar.dalloc((size_t)m * m);
    double* Xc = ar.dalloc((size_t)n * m);
    double* BX = ar.dalloc((size_t)n * m);
    double* Qc = ar.dalloc((size_t)m * m);
    double* lc = ar.dalloc(std::max(m, 64));
    std::vector<CopyDesc> dx;
    for (int q = 0; q < m; ++q) dx.push_back({(long long)c[q] * n, (long long)q * n, n, n, n, 1});
    copy_blocks(X, Xc, dx, ar, s);
    {
      GemmBatch g;
      g.m = n; g.n = m; g.k = n;
      g.A = B; g.lda = ldb; g.B = Xc; g.ldb = n; g.C = BX; g.ldc = n;
      dgemm(g, s);
      GemmBatch h;
      h.transA = 1;
      h.m = m; h.n = m; h.k = n;
      h.A = Xc; h.lda = n; h.B = BX; h.ldb = n; h.C = Sc; h.ldc = m;
      dgemm(h, s);
    }
    symmetrize(1, m, Sc, m, 0, s);
    if (m <= 64) {
      std::vector<int> sz = {m};
      int* d_sz = static_cast<int*>(ar.alloc(sizeof(int)));
      h2d(d_sz, sz.data(), sizeof(int), s);
      jacobi_batched(1, d_sz, Sc, m, (long long)m * m, Qc, m, (long long)m * m, lc, s);
    } else {
      double lo = lh[c.front()], hi = lh[c.back()];
      const double pad = std::max(4.0 * delta, 1e-300);
      ZoloEigArgs ea;
      ea.n = m;
      ea.B = Sc; ea.ldb = m;
      ea.lo = lo - pad; ea.hi = hi + pad;
      ea.V = Qc; ea.ldv = m;
      ea.lam = lc;
      zolo_eig(ea, ar, s);
    }
    // X(:, c) = Xc Qc
    double* Xr = ar.dalloc((size_t)n * m);
    GemmBatch g;
    g.m = n; g.n = m; g.k = m;
    g.A = Xc; g.lda = n; g.B = Qc; g.ldb = m; g.C = Xr; g.ldc = n;
    dgemm(g, s);
    std::vector<CopyDesc> back;
    for (int q = 0; q < m; ++q) back.push_back({(long long)q * n, (long long)c[q] * n, n, n, n, 1});
    copy_blocks(Xr, X, back, ar, s);
    std::vector<double> lch(m);
    d2h(lch.data(), lc, m * sizeof(double), s);
    for (int q = 0; q < m; ++q) lh[c[q]] = lch[q];
  }
  // ascending order
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return lh[x] < lh[y]; });
  {
    std::vector<CopyDesc> cv;
    std::vector<double> ls(n);
    for (int j = 0; j < n; ++j) {
      cv.push_back({(long long)ord[j] * n, (long long)j * n, n, n, n, 1});
      ls[j] = lh[ord[j]];
    }
    copy_blocks(X, Xn, cv, ar, s);
    copy_scale(1, n, n, 1.0, Xn, n, 0, X, n, 0, s);
    h2d(lam, ls.data(), n * sizeof(double), s);
  }
  return res;
}

}  // namespace zcsd
