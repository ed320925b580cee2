// CS decomposition of a complex partial isometry (the paper's setting,
// A_i in C^{n x n}; Sec. 1 and Theorem 2.1) through its real embedding.
//
// A complex matrix X + iY acts on R^{2n} as [X -Y; Y X], and that map keeps
// products, (conjugate) transposes and unitarity.  The embedding of
// A = [A1; A2] is a real partial isometry of twice the rank whose angles are
// those of A, each twice: a complex singular triple (u1, u2, v; theta) gives
// the real ones built from [Re v; Im v] and from J [Re v; Im v], where
// J = [0 -I; I 0] is multiplication by i.  Algorithm 1 / 3 therefore runs
// unchanged on the embedding (the real path at size 2n), and the complex
// factors are read back from it:
//   1. the 2r real angles come in equal pairs; runs of them closer than a
//      pairing gap form clusters, a complex multiplicity m giving 2m;
//   2. a two-column cluster spans one complex line: its first real column
//      [a; b] gives the complex column a + ib of V1 (and U1, U2 from the
//      real columns the decomposition pairs with it, so that the phase is
//      the same);
//   3. a larger cluster with real basis X (2n x 2m, columns of V1) spans m
//      complex dimensions, but its columns need not come in J-pairs.
//      M = X^T J X is then orthogonal and skew (J maps the span onto itself),
//      and T = D + M^T D M, with D a fixed diagonal of distinct values,
//      commutes with M, so that its eigenvectors come in pairs (q, M q) of
//      one eigenvalue; one vector of each pair, Q1 (2m x m), gives X Q1 whose
//      columns are orthonormal and orthogonal to their images under J, that
//      is complex-orthonormal.  The same Q1 applied to the cluster's U1 and
//      U2 columns keeps U_i = W_i V1;
//   4. eigenvectors of neighbouring angles (gap g) mix at the u/g level
//      inside the real decomposition, which costs complex orthogonality at
//      that level; Newton-Schulz steps V <- V (3 I - V^* V) / 2 on V1, with
//      the same right factor on U1 and U2 (so that U_i = W_i V1 still holds),
//      restore it.  Each step is computed on the embedded columns [V, J V],
//      whose products are those of the complex ones;
//   5. the computed real polar factor W_i commutes with J only up to about
//      u / sigma on the singular vectors of A_i with small singular values
//      sigma (cos theta for U1, sin theta for U2), so U1 and U2 get their own
//      correction steps next, from their own Gram matrices.  A symmetric step
//      would move a well-determined column by u / sigma_j times a poorly
//      determined one; the first-order inverse Cholesky factor
//      I - diag(E)/2 - triu(E, 1) of G = I + E instead corrects each column
//      only by those of larger sigma, which changes A_i's reconstruction by
//      O(u).  Columns with sigma below 2^-46, which A does not determine at
//      all, are replaced by any orthonormal completion: complex Gaussian
//      columns projected off the others and orthonormalised through the
//      eigendecomposition of their embedded Gram matrix;
//   6. the angles follow from the final factors as in Algorithm 1,
//      C_kk = Re(u1_k^* A1 v_k) and S_kk = Re(u2_k^* A2 v_k).
// Twice the flops of complex arithmetic, but every step runs on the tested
// real kernels.
#include <algorithm>
#include <cmath>
#include <initializer_list>
#include <vector>

#include "zcsd_api_guard.h"
#include "zcsd_eig.h"
#include "zcsd_internal.h"
#include "zcsd_la.h"

namespace zcsd {
namespace {

// E (2m x 2n, ld 2m) = [Re A  -Im A; Im A  Re A], A m x n interleaved complex (ld lda)
__global__ void complex_embed_kernel(int m, int n, const double* __restrict__ A, long long lda,
                                     double* __restrict__ E) {
  const long long M2 = 2LL * m, total = M2 * 2 * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e % M2), c = (int)(e / M2);
    const long long src = 2 * ((r % m) + (long long)(c % n) * lda);
    const double re = A[src], im = A[src + 1];
    const bool top = r < m, left = c < n;
    E[e] = (top == left) ? re : (top ? -im : im);
  }
}

// Y(:, k) = R(:, col[k]) (both with `rows` rows and ld rows), k = blockIdx.y
__global__ void gather_columns_kernel(long long rows, const double* __restrict__ R,
                                      const int* __restrict__ col, double* __restrict__ Y) {
  const int k = blockIdx.y;
  const double* src = R + (long long)col[k] * rows;
  double* dst = Y + (long long)k * rows;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < rows;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// P = [Y, J Y]: Y is 2h x r (ld 2h), P is 2h x 2r (ld 2h), J [a; b] = [-b; a]
__global__ void with_j_image_kernel(int h, int r, const double* __restrict__ Y,
                                    double* __restrict__ P) {
  const long long N = 2LL * h;
  const int k = blockIdx.y;
  const double* y = Y + (long long)k * N;
  double* p0 = P + (long long)k * N;
  double* p1 = P + (long long)(r + k) * N;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    p0[i] = y[i];
    p1[i] = (i < h) ? -y[i + h] : y[i - h];
  }
}

// complex column k of Z (h rows, interleaved, ld ldz) = Y(0:h, j) + i Y(h:2h, j)
// with j = perm[k] for k < r, zero for k >= r; Y is 2h x r (ld 2h); k = blockIdx.y
__global__ void to_complex_kernel(int h, int r, const double* __restrict__ Y,
                                  const int* __restrict__ perm, double* __restrict__ Z,
                                  long long ldz) {
  const int k = blockIdx.y;
  double* z = Z + 2LL * k * ldz;
  const double* y = Y + 2LL * (k < r ? perm[k] : 0) * h;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < h; i += gridDim.x * blockDim.x) {
    z[2 * i] = k < r ? y[i] : 0.0;
    z[2 * i + 1] = k < r ? y[h + i] : 0.0;
  }
}

// out[j] = X(:, j) . Y(:, j), columns of `rows` entries (ld rows); j = blockIdx.x
__global__ void column_dots_kernel(long long rows, const double* __restrict__ X,
                                   const double* __restrict__ Y, double* __restrict__ out) {
  __shared__ double part[256];
  const long long off = (long long)blockIdx.x * rows;
  double acc = 0.0;
  for (long long i = threadIdx.x; i < rows; i += blockDim.x) acc += X[off + i] * Y[off + i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

// In place on G (2c x c, ld 2c), which holds [Re E; Im E] for a complex
// Hermitian E (c x c): the factor H = [Re F; Im F] with F = I - E/2 (mode 0),
// I - diag(E)/2 - triu(E, 1) (mode 1) or I - diag(E)/2 - tril(E, -1) (mode 2)
__global__ void correction_factor_kernel(int c, int mode, double* __restrict__ G) {
  const long long total = 2LL * c * c;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int row = (int)(e % (2LL * c)), col = (int)(e / (2LL * c));
    const bool re = row < c;
    const int i = re ? row : row - c;
    const double g = G[e];
    double h;
    if (i == col) {
      h = re ? 1.0 - 0.5 * g : (mode == 0 ? -0.5 * g : 0.0);
    } else {
      const bool keep = mode == 0 || (mode == 1 ? i < col : i > col);
      h = keep ? (mode == 0 ? -0.5 * g : -g) : 0.0;
    }
    G[e] = h;
  }
}

// splitmix64 (Steele, Lea and Flood), the output function used as a hash
__device__ inline unsigned long long splitmix64(unsigned long long z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// X[e] ~ N(0, 1) by Box-Muller from two hashed uniforms
__global__ void gaussian_fill_kernel(long long total, unsigned long long seed,
                                     double* __restrict__ X) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const double u1 = ((double)(splitmix64(seed + 2ULL * e) >> 11) + 0.5) * 0x1p-53;
    const double u2 = (double)(splitmix64(seed + 2ULL * e + 1ULL) >> 11) * 0x1p-53;
    X[e] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
  }
}

// out(:, j) = Q(:, j) / sqrt(max(lam_j, floor))  (p x p, ld p)
__global__ void scale_columns_kernel(int p, const double* __restrict__ Q,
                                     const double* __restrict__ lam, double floor,
                                     double* __restrict__ out) {
  const long long total = (long long)p * p;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x)
    out[e] = Q[e] * rsqrt(fmax(lam[e / p], floor));
}

// P = diag(d) M (p x p, ld p)
__global__ void row_scale_kernel(int p, const double* __restrict__ d, const double* __restrict__ M,
                                 double* __restrict__ P) {
  const long long total = (long long)p * p;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x)
    P[e] = d[e % p] * M[e];
}

// T(i, i) += d(i)  (p x p, ld p)
__global__ void add_diag_vec_kernel(int p, const double* __restrict__ d, double* __restrict__ T) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p) T[(long long)i * p + i] += d[i];
}

unsigned grid_for(long long work) {
  return (unsigned)std::max<long long>(1, std::min<long long>((work + 255) / 256, 8192));
}

void gemm(int ta, int tb, int m, int n, int k, double alpha, const double* A, long long lda,
          const double* B, long long ldb, double beta, double* C, long long ldc, hipStream_t s) {
  GemmBatch g;
  g.transA = ta;
  g.transB = tb;
  g.m = m;
  g.n = n;
  g.k = k;
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  g.C = C;
  g.ldc = ldc;
  g.alpha = alpha;
  g.beta = beta;
  dgemm(g, s);
}

// p distinct values in [1, 2): the golden-ratio (Kronecker) sequence
std::vector<double> distinct_diagonal(int p) {
  std::vector<double> d(p);
  const double phi = 0.6180339887498949;
  for (int i = 0; i < p; ++i) d[i] = 1.0 + std::fmod(0.5 + phi * (i + 1), 1.0);
  return d;
}

// doubles held at once: the embeddings, the real factors, the selected
// columns and the angles for the whole call; then, one phase at a time, the
// blocks' QR reduction (rectangular blocks), the cluster matrices (up to
// four (2n)^2), the re-orthonormalisation and completion temporaries and the
// angle products (all below 8 (2n)^2 + 6 (2 max(m1, m2)) (2n)); plus the real
// path's workspace at 2n and the QR workspace
size_t complex_workspace_bytes(int m1, int m2, int n) {
  const long long N = 2LL * n, NN = N * N, mx = 2LL * std::max(m1, m2);
  const long long rows = 2LL * m1 + 2LL * m2 + N;
  const long long held = (2LL * m1 + 2LL * m2) * N + rows * N + rows * n + 2 * N;
  const long long qr = (m1 == n && m2 == n) ? 0 : (2LL * m1 + 2LL * m2) * N + 4 * NN + mx * N;
  const long long phase = std::max(qr, 8 * NN + 6 * mx * N);
  return csd_workspace_bytes((int)N) + (size_t)(held + phase) * sizeof(double) +
         ((m1 == n && m2 == n) ? 0 : qr_work_bytes(QRShape::General, 1, (int)mx, (int)N, 32)) +
         ((size_t)64 << 20);
}

}  // namespace
}  // namespace zcsd

using namespace zcsd;

namespace zcsd {
namespace {

// Algorithm 1 / 3 on the real embedding of complex A1 (m1 x n), A2 (m2 x n),
// m1, m2 >= n, and the read-back of the complex factors (see the top of the file)
void complex_csd(zcsd_handle* handle, int m1, int m2, int n, const double* d_A1, long long lda1,
                 const double* d_A2, long long lda2, double* d_U1, long long ldu1, double* d_U2,
                 long long ldu2, double* d_V1, long long ldv1, double* d_theta, const zcsd_opts& o,
                 zcsd_info* info) {
  ZCSD_REQUIRE(o.prec == ZCSD_FP64, "zcsd: complex input is computed in the FP64 mode only");
  ZCSD_HIP(hipSetDevice(handle->device));
  const int N = 2 * n;
  const long long NN = (long long)N * N;
  // factors q = 0 (U1), 1 (U2), 2 (V1): rows of the real factor, half of them
  const long long rows[3] = {2LL * m1, 2LL * m2, N};
  const int half[3] = {m1, m2, n};
  Arena& ar = handle->arena;
  ar.reset();
  ar.reserve(complex_workspace_bytes(m1, m2, n));
  hipStream_t s = handle->stream;
  double* E[2] = {ar.dalloc((size_t)rows[0] * N), ar.dalloc((size_t)rows[1] * N)};
  double* R[3];  // the real factors (rows[q] x N), later scratch for [Y, JY]
  double* Y[3];  // the selected columns (rows[q] x n)
  for (int q = 0; q < 3; ++q) R[q] = ar.dalloc((size_t)rows[q] * N);
  for (int q = 0; q < 3; ++q) Y[q] = ar.dalloc((size_t)rows[q] * n);
  double* th = ar.dalloc(N);
  const double* A[2] = {d_A1, d_A2};
  const long long lda[2] = {lda1, lda2};
  for (int i = 0; i < 2; ++i) {
    hipLaunchKernelGGL(complex_embed_kernel, dim3(grid_for(rows[i] * N)), dim3(256), 0, s, half[i],
                       n, A[i], lda[i], E[i]);
    ZCSD_CHECK_LAUNCH();
  }
  bool repaired = false;
  int rank2;
  if (m1 == n && m2 == n) {
    rank2 = csd_single_member(N, E[0], E[1], R[0], R[1], R[2], th, o, ar, s, &repaired);
  } else {
    // rectangular blocks: E_i = Q_i R_i, the square path on [R_1; R_2] (a
    // partial isometry with the same angles and V1), U_i = Q_i U_i'
    ArenaScope sc(ar);
    double* Qt[2] = {ar.dalloc((size_t)rows[0] * N), ar.dalloc((size_t)rows[1] * N)};
    double* Rt = ar.dalloc(2 * (size_t)NN);
    double* Up = ar.dalloc(2 * (size_t)NN);
    for (int i = 0; i < 2; ++i) tall_qr((int)rows[i], N, E[i], rows[i], Qt[i], Rt + i * NN, ar, s);
    rank2 = csd_single_member(N, Rt, Rt + NN, Up, Up + NN, R[2], th, o, ar, s, &repaired);
    for (int i = 0; i < 2; ++i)
      gemm(0, 0, (int)rows[i], N, N, 1.0, Qt[i], rows[i], Up + i * NN, N, 0.0, R[i], rows[i], s);
  }
  if (rank2 % 2) throw NumError(ZCSD_ENOCONV, "zcsd: odd rank of the real embedding");
  const int r = rank2 / 2;
  std::vector<double> thh(std::max(1, rank2));
  if (rank2) d2h(thh.data(), th, rank2 * sizeof(double), s);

  // 1. clusters of real angles: consecutive gaps within the pairing gap
  const double pair_gap = 0x1p-40 * (1.0 + N / 1024.0);
  struct Cluster { int begin, end; };
  std::vector<Cluster> cl;
  for (int j = 0; j < rank2;) {
    int e = j + 1;
    while (e < rank2 && thh[e] - thh[e - 1] <= pair_gap) ++e;
    if ((e - j) % 2)
      throw NumError(ZCSD_ENOCONV, "zcsd: an angle of the real embedding without its pair");
    cl.push_back({j, e});
    j = e;
  }
  // 2. the first real column of every pair
  std::vector<int> col(std::max(1, r), 0);
  {
    int k = 0;
    for (const Cluster& c : cl)
      for (int j = c.begin; j < c.end; j += 2) col[k++] = j;
  }
  if (r > 0) {
    int* d_col = ar.ialloc(r);
    h2d(d_col, col.data(), r * sizeof(int), s);
    for (int q = 0; q < 3; ++q) {
      hipLaunchKernelGGL(gather_columns_kernel, dim3(grid_for(rows[q]), r), dim3(256), 0, s,
                         rows[q], R[q], d_col, Y[q]);
      ZCSD_CHECK_LAUNCH();
    }
  }
  // 3. clusters of complex multiplicity m > 1: a complex-orthonormal basis
  {
    int k = 0;
    for (const Cluster& c : cl) {
      const int p = c.end - c.begin, m = p / 2;
      if (m > 1) {
        ArenaScope scope(ar);
        const long long pp = (long long)p * p;
        double* M = ar.dalloc(pp);
        double* P = ar.dalloc(pp);
        double* T = ar.dalloc(pp);
        double* Q = ar.dalloc(pp);
        double* lam = ar.dalloc(p);
        double* dd = ar.dalloc(p);
        const double* X = R[2] + (long long)c.begin * N;  // V1 columns of the cluster
        // M = X^T J X = Xb^T Xt - Xt^T Xb  (X = [Xt; Xb])
        gemm(1, 0, p, p, n, 1.0, X + n, N, X, N, 0.0, M, p, s);
        gemm(1, 0, p, p, n, -1.0, X, N, X + n, N, 1.0, M, p, s);
        // T = M^T (D M) + D
        const std::vector<double> d = distinct_diagonal(p);
        h2d(dd, d.data(), p * sizeof(double), s);
        hipLaunchKernelGGL(row_scale_kernel, dim3(grid_for(pp)), dim3(256), 0, s, p, dd, M, P);
        ZCSD_CHECK_LAUNCH();
        gemm(1, 0, p, p, p, 1.0, M, p, P, p, 0.0, T, p, s);
        hipLaunchKernelGGL(add_diag_vec_kernel, dim3((p + 255) / 256), dim3(256), 0, s, p, dd, T);
        ZCSD_CHECK_LAUNCH();
        symmetrize(1, p, T, p, 0, s);
        // D and M^T D M both have their spectrum in [1, 2]
        ZoloEigArgs ea;
        ea.n = p;
        ea.B = T;
        ea.ldb = p;
        ea.lo = 1.99;
        ea.hi = 4.01;
        ea.V = Q;
        ea.ldv = p;
        ea.lam = lam;
        ea.n_leaf = o.n_leaf;
        ea.eps = o.eps;
        ea.tol = o.tol;
        ea.measure_offblock = false;
        zolo_eig(ea, ar, s);
        // one eigenvector of each pair: columns 0, 2, 4, ... (ld 2p)
        for (int q = 0; q < 3; ++q)
          gemm(0, 0, (int)rows[q], m, p, 1.0, R[q] + (long long)c.begin * rows[q], rows[q], Q,
               2LL * p, 0.0, Y[q] + (long long)k * rows[q], rows[q], s);
      }
      k += m;
    }
  }
  // 4. complex orthonormality of the factors (items 4 and 5 above)
  if (r > 0) {
    // angle of each complex column: its cluster's mean (ascending)
    std::vector<double> thk(r);
    {
      int k = 0;
      for (const Cluster& c : cl) {
        double mean = 0.0;
        for (int j = c.begin; j < c.end; ++j) mean += thh[j];
        mean /= (c.end - c.begin);
        for (int j = c.begin; j < c.end; j += 2) thk[k++] = mean;
      }
    }
    // columns whose U1 (cos below tau: a suffix) or U2 (sin below tau: a
    // prefix) column A leaves undetermined
    const double tau = 0x1p-46;
    int t1 = 0, t2 = 0;
    for (int k = 0; k < r; ++k) {
      if (std::cos(thk[k]) < tau) ++t1;
      if (std::sin(thk[k]) < tau) ++t2;
    }
    ArenaScope scope(ar);
    double* G = ar.dalloc(2LL * r * r);  // 2 cnt x cnt, ld 2 cnt
    double* ss = ar.dalloc(1);
    // Correction steps on columns [c0, c0 + cnt) of the factors in `apply`,
    // from the complex Gram matrix of factor gq on those columns, G = I + E:
    // mode 0 multiplies by I - E/2 (Newton-Schulz), mode 1 by
    // I - diag(E)/2 - triu(E, 1) and mode 2 by I - diag(E)/2 - tril(E, -1)
    // (first-order inverse Cholesky factors: a column is corrected only by
    // the columns before it, resp. after it).  Returns the last ||E||_F, or 0
    // once a step was taken from ||E||_F < 1e-8 (leaving O(||E||^2)).
    auto correct = [&](int gq, std::initializer_list<int> apply, int c0, int cnt, int mode,
                       int max_steps) {
      double eta = 0.0;
      const long long ldg = 2LL * cnt;
      for (int step = 0; step < max_steps; ++step) {
        for (int q : apply) {
          hipLaunchKernelGGL(with_j_image_kernel, dim3(grid_for(rows[q]), cnt), dim3(256), 0, s,
                             half[q], cnt, Y[q] + (long long)c0 * rows[q], R[q]);
          ZCSD_CHECK_LAUNCH();
        }
        gemm(1, 0, 2 * cnt, cnt, (int)rows[gq], 1.0, R[gq], rows[gq],
             Y[gq] + (long long)c0 * rows[gq], rows[gq], 0.0, G, ldg, s);
        add_diag(1, cnt, -1.0, G, ldg, 0, s);
        sumsq(1, 2 * cnt, cnt, G, ldg, 0, ss, ar, s);
        double eta2 = 0.0;
        d2h(&eta2, ss, sizeof(double), s);
        if (!std::isfinite(eta2)) throw NumError(ZCSD_ENOCONV, "zcsd: non-finite factor");
        eta = std::sqrt(eta2);
        hipLaunchKernelGGL(correction_factor_kernel, dim3(grid_for(2LL * cnt * cnt)), dim3(256), 0,
                           s, cnt, mode, G);
        ZCSD_CHECK_LAUNCH();
        for (int q : apply)
          gemm(0, 0, (int)rows[q], cnt, 2 * cnt, 1.0, R[q], rows[q], G, ldg, 0.0,
               Y[q] + (long long)c0 * rows[q], rows[q], s);
        if (eta < 1e-8) return 0.0;
      }
      return eta;
    };
    // any complex-orthonormal basis of t columns orthogonal to the cnt
    // columns at cg of factor q, written at cb: the polar factor of the
    // projection of complex Gaussian columns, through the eigendecomposition
    // of the embedded Gram matrix (a function of it, hence itself embedded)
    auto complete = [&](int q, int cb, int t, int cg, int cnt) {
      ArenaScope sc(ar);
      const long long rq = rows[q];
      double* Om = ar.dalloc((size_t)rq * t);
      hipLaunchKernelGGL(gaussian_fill_kernel, dim3(grid_for(rq * t)), dim3(256), 0, s, rq * t,
                         0x5eedULL + 977ULL * q, Om);
      ZCSD_CHECK_LAUNCH();
      if (cnt > 0) {
        double* Tm = ar.dalloc(2LL * cnt * t);
        hipLaunchKernelGGL(with_j_image_kernel, dim3(grid_for(rq), cnt), dim3(256), 0, s, half[q],
                           cnt, Y[q] + (long long)cg * rq, R[q]);
        ZCSD_CHECK_LAUNCH();
        for (int pass = 0; pass < 2; ++pass) {
          gemm(1, 0, 2 * cnt, t, (int)rq, 1.0, R[q], rq, Om, rq, 0.0, Tm, 2LL * cnt, s);
          gemm(0, 0, (int)rq, t, 2 * cnt, -1.0, R[q], rq, Tm, 2LL * cnt, 1.0, Om, rq, s);
        }
      }
      const int p = 2 * t;
      const long long pp = (long long)p * p;
      double* PJ = ar.dalloc((size_t)rq * p);
      double* G2 = ar.dalloc(pp);
      double* Q = ar.dalloc(pp);
      double* Qs = ar.dalloc(pp);
      double* lam = ar.dalloc(p);
      double* Mt = ar.dalloc((size_t)p * t);
      double* nrm = ar.dalloc(1);
      hipLaunchKernelGGL(with_j_image_kernel, dim3(grid_for(rq), t), dim3(256), 0, s, half[q], t, Om,
                         PJ);
      ZCSD_CHECK_LAUNCH();
      gemm(1, 0, p, p, (int)rq, 1.0, PJ, rq, PJ, rq, 0.0, G2, p, s);
      symmetrize(1, p, G2, p, 0, s);
      sumsq(1, p, p, G2, p, 0, nrm, ar, s);
      double f2 = 0.0;
      d2h(&f2, nrm, sizeof(double), s);
      const double hi = 1.01 * std::sqrt(f2) + 1e-300;
      if (!std::isfinite(hi)) throw NumError(ZCSD_ENOCONV, "zcsd: non-finite completion");
      ZoloEigArgs ea;
      ea.n = p;
      ea.B = G2;
      ea.ldb = p;
      ea.lo = -0.01 * hi;
      ea.hi = hi;
      ea.V = Q;
      ea.ldv = p;
      ea.lam = lam;
      ea.n_leaf = o.n_leaf;
      ea.eps = o.eps;
      ea.tol = o.tol;
      ea.measure_offblock = false;
      zolo_eig(ea, ar, s);
      // M(:, 0:t) = Q diag(lam)^(-1/2) Q(0:t, :)^T
      hipLaunchKernelGGL(scale_columns_kernel, dim3(grid_for(pp)), dim3(256), 0, s, p, Q, lam,
                         1e-30 * hi, Qs);
      ZCSD_CHECK_LAUNCH();
      gemm(0, 1, p, t, p, 1.0, Qs, p, Q, p, 0.0, Mt, p, s);
      gemm(0, 0, (int)rq, t, p, 1.0, PJ, rq, Mt, p, 0.0, Y[q] + (long long)cb * rq, rq, s);
    };
    // V1 (and U1, U2 with V1's factor, which keeps U_i = W_i V1)
    if (correct(2, {0, 1, 2}, 0, r, 0, 3) > 0.0)
      throw NumError(ZCSD_ENOCONV, "zcsd: V1 did not become orthonormal");
    // U1 and U2 on their own, each column corrected only by the columns of
    // larger cos (U1) or sin (U2): those are at least as well determined
    if (r - t1 > 0 && correct(0, {0}, 0, r - t1, 1, 4) > 0.0)
      throw NumError(ZCSD_ENOCONV, "zcsd: U1 did not become orthonormal");
    if (r - t2 > 0 && correct(1, {1}, t2, r - t2, 2, 4) > 0.0)
      throw NumError(ZCSD_ENOCONV, "zcsd: U2 did not become orthonormal");
    if (t1 > 0) {
      complete(0, r - t1, t1, 0, r - t1);
      if (correct(0, {0}, 0, r, 0, 3) > 0.0)
        throw NumError(ZCSD_ENOCONV, "zcsd: U1 did not become orthonormal");
    }
    if (t2 > 0) {
      complete(1, 0, t2, t2, r - t2);
      if (correct(1, {1}, 0, r, 0, 3) > 0.0)
        throw NumError(ZCSD_ENOCONV, "zcsd: U2 did not become orthonormal");
    }
  }
  // 5. angles from the final factors, C_kk = Re(u1_k^* A1 v_k) and
  //    S_kk = Re(u2_k^* A2 v_k): Algorithm 1's diagonals of V1^* H_i V1,
  //    since U_i^* A_i = V1^* W_i^* W_i H_i = V1^* H_i.  For embedded
  //    columns that is the real dot product [Re u; Im u] . (embedded A_i)
  //    [Re v; Im v]; columns in ascending order of theta
  std::vector<double> thc(n, 0.0);
  std::vector<int> perm(n);
  for (int k = 0; k < n; ++k) perm[k] = k;
  if (r > 0) {
    ArenaScope scope(ar);
    double* P = ar.dalloc((size_t)std::max(rows[0], rows[1]) * r);
    double* cs = ar.dalloc(2LL * r);
    for (int i = 0; i < 2; ++i) {
      gemm(0, 0, (int)rows[i], r, N, 1.0, E[i], rows[i], Y[2], N, 0.0, P, rows[i], s);
      hipLaunchKernelGGL(column_dots_kernel, dim3(r), dim3(256), 0, s, rows[i], Y[i], P,
                         cs + (long long)i * r);
      ZCSD_CHECK_LAUNCH();
    }
    std::vector<double> h(2 * (size_t)r);
    d2h(h.data(), cs, h.size() * sizeof(double), s);
    for (int k = 0; k < r; ++k)
      thc[k] = std::min(std::max(std::atan2(h[r + k], h[k]), 0.0), 0.5 * M_PI);
    std::stable_sort(perm.begin(), perm.begin() + r, [&](int a, int b) { return thc[a] < thc[b]; });
    std::vector<double> sorted(n, 0.0);
    for (int k = 0; k < r; ++k) sorted[k] = thc[perm[k]];
    thc.swap(sorted);
  }
  // 6. complex columns
  int* d_perm = ar.ialloc(n);
  h2d(d_perm, perm.data(), n * sizeof(int), s);
  double* outs[3] = {d_U1, d_U2, d_V1};
  const long long lds[3] = {ldu1, ldu2, ldv1};
  for (int q = 0; q < 3; ++q) {
    hipLaunchKernelGGL(to_complex_kernel, dim3(grid_for(half[q]), n), dim3(256), 0, s, half[q], r,
                       Y[q], d_perm, outs[q], lds[q]);
    ZCSD_CHECK_LAUNCH();
  }
  h2d(d_theta, thc.data(), n * sizeof(double), s);
  ZCSD_HIP(hipStreamSynchronize(s));
  if (info) {
    *info = zcsd_info{};
    info->rank = r;
    info->repair = repaired ? 1 : 0;
  }
}

}  // namespace
}  // namespace zcsd

using namespace zcsd;

extern "C" zcsd_status zcsd_zcsd(zcsd_handle* handle, int n, const double* d_A1, int lda1,
                                 const double* d_A2, int lda2, double* d_U1, int ldu1,
                                 double* d_U2, int ldu2, double* d_V1, int ldv1, double* d_theta,
                                 const zcsd_opts* opts, zcsd_info* info) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(n >= 1 && n <= 32767, "zcsd: n must lie in [1, 32767]");
    ZCSD_REQUIRE(d_A1 && d_A2 && d_U1 && d_U2 && d_V1 && d_theta, "zcsd: NULL pointer");
    ZCSD_REQUIRE(lda1 >= n && lda2 >= n && ldu1 >= n && ldu2 >= n && ldv1 >= n,
                 "zcsd: leading dimension < n");
    zcsd_opts o;
    zcsd_default_opts(&o);
    if (opts) o = *opts;
    complex_csd(handle, n, n, n, d_A1, lda1, d_A2, lda2, d_U1, ldu1, d_U2, ldu2, d_V1, ldv1,
                d_theta, o, info);
  });
}

extern "C" zcsd_status zcsd_zcsd_mn(zcsd_handle* handle, int m1, int m2, int n,
                                    const double* d_A1, int lda1, const double* d_A2, int lda2,
                                    double* d_U1, int ldu1, double* d_U2, int ldu2, double* d_V1,
                                    int ldv1, double* d_theta, const zcsd_opts* opts,
                                    zcsd_info* info) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(n >= 1 && m1 >= n && m2 >= n && m1 <= 32767 && m2 <= 32767,
                 "zcsd_mn: need 1 <= n <= m1, m2 <= 32767");
    ZCSD_REQUIRE(d_A1 && d_A2 && d_U1 && d_U2 && d_V1 && d_theta, "zcsd_mn: NULL pointer");
    ZCSD_REQUIRE(lda1 >= m1 && lda2 >= m2 && ldu1 >= m1 && ldu2 >= m2 && ldv1 >= n,
                 "zcsd_mn: leading dimension too small");
    zcsd_opts o;
    zcsd_default_opts(&o);
    if (opts) o = *opts;
    complex_csd(handle, m1, m2, n, d_A1, lda1, d_A2, lda2, d_U1, ldu1, d_U2, ldu2, d_V1, ldv1,
                d_theta, o, info);
  });
}
