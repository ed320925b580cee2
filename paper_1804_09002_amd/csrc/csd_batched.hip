// Batched Zolo-csd over problems of different sizes (packed, ragged layout).
//
// Problems are grouped into size classes; inside a class every problem is
// embedded in the class size N with padding that cannot mix with its
// spectrum, and the class runs through the batched kernels of the single
// path as one problem set:
//   polar (Algorithm 1): X = diag(A_i, I).  The padding has singular
//       value 1, which Z maps to 1, so W = diag(W_i, I), H = diag(H_i, I)
//       (up to rounding-level coupling that is discarded);
//   B: built on the real n x n part, the padding set to exactly 3 I
//       with exactly zero coupling.  The real spectrum lies in [-1, 1] (plus
//       mu = 2 on the null space of a rank-deficient input, Alg. 3), so the
//       padding is an isolated eigenvalue and every eigenvector of the real
//       part has zero padding rows up to rounding;
//   eig: one batched Zolo-eig over the class;
//   selection: the eigenpairs with lambda <= 2 (full rank) or <= (1 + mu)/2
//       (Algorithm 3, null space at mu) are the real ones; the padding at 3
//       is dropped the same way;
//   assembly (Algorithm 1, Remark (iii)): U_i = W_i V1, c = diag(V1^T H1 V1),
//       s = diag(V1^T H2 V1), theta = atan2(s, c), sorted per problem.
// Full-rank and rank-deficient problems of a class are separate sub-batches
// (the latter use the modified Zolo-pd with l = eps, r = 8).
#include <algorithm>
#include <cmath>
#include <exception>
#include <map>
#include <numeric>
#include <thread>
#include <vector>

#include "zcsd_api_guard.h"
#include "zcsd_eig.h"
#include "zcsd_internal.h"
#include "zcsd_la.h"
#include "zcsd_zolo.h"

namespace zcsd {

// ss[2k + i] = ||A_i of problem k||_F^2, one workgroup per (matrix, problem)
__global__ void ragged_sumsq_kernel(const double* __restrict__ A1, const double* __restrict__ A2,
                                    const long long* __restrict__ off, const int* __restrict__ nk,
                                    double* ss) {
  const int k = blockIdx.x, which = blockIdx.y;
  const double* A = (which == 0 ? A1 : A2) + off[k];
  const long long tot = (long long)nk[k] * nk[k];
  double acc = 0.0;
  for (long long e = threadIdx.x; e < tot; e += blockDim.x) acc += A[e] * A[e];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) ss[2 * k + which] = red[0];
}

// X[2q + i] = diag(A_i of member q, I_{N - n_q})  (N x N, ld N)
__global__ void pad_pack_kernel(int N, const double* __restrict__ A1, const double* __restrict__ A2,
                                const long long* __restrict__ off, const int* __restrict__ nq,
                                double* X) {
  const int q = blockIdx.y >> 1, which = blockIdx.y & 1;
  const double* A = (which == 0 ? A1 : A2) + off[q];
  const int n = nq[q];
  const long long NN = (long long)N * N;
  double* Xq = X + (long long)blockIdx.y * NN;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < NN;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % N), j = (int)(e / N);
    Xq[e] = (i < n && j < n) ? A[i + (long long)j * n] : ((i == j) ? 1.0 : 0.0);
  }
}

// B_q = sym(H2 - H1) + mu (I - sym(G)) on the real part (G = A^T A when mu != 0),
// 3 I on the padding, zero coupling
__global__ void build_b_kernel(int N, const double* __restrict__ H, const double* __restrict__ G,
                               double mu, const int* __restrict__ nq, double* B) {
  const int q = blockIdx.y;
  const int n = nq[q];
  const long long NN = (long long)N * N;
  const double* H1 = H + 2LL * q * NN;
  const double* H2 = H1 + NN;
  const double* Gq = G ? G + q * NN : nullptr;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < NN;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % N), j = (int)(e / N);
    double v;
    if (i < n && j < n) {
      const long long t = j + (long long)i * N;
      v = 0.5 * ((H2[e] - H1[e]) + (H2[t] - H1[t]));
      if (Gq) v += mu * (((i == j) ? 1.0 : 0.0) - 0.5 * (Gq[e] + Gq[t]));
    } else {
      v = (i == j) ? 3.0 : 0.0;
    }
    B[q * NN + e] = v;
  }
}

// Y = a X + b Y over `total` contiguous elements
__global__ void axpby_flat_kernel(long long total, double a, const double* __restrict__ X, double b,
                                  double* Y) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x)
    Y[e] = a * X[e] + b * Y[e];
}

// zero the columns j >= r_q of U (both polars of member q), N x N blocks
__global__ void mask_cols_kernel(int N, double* U, const int* __restrict__ rq) {
  const int b = blockIdx.y;  // matrix index 2q + i
  const int r = rq[b >> 1];
  const long long NN = (long long)N * N;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < NN;
       e += (long long)gridDim.x * blockDim.x)
    if ((int)(e / N) >= r) U[b * NN + e] = 0.0;
}

// cs[b][j] = sum_{i < n_q} V_q(i, j) T_b(i, j), b = 2q + i; one workgroup per (j, b)
__global__ void coldot_ragged_kernel(int N, const double* __restrict__ V, const double* __restrict__ T,
                                     const int* __restrict__ nq, double* cs) {
  const int j = blockIdx.x, b = blockIdx.y;
  const int n = nq[b >> 1];
  const long long NN = (long long)N * N;
  const double* v = V + (long long)(b >> 1) * NN + (long long)j * N;
  const double* t = T + (long long)b * NN + (long long)j * N;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += v[i] * t[i];
  __shared__ double red[64];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) cs[(long long)b * N + j] = red[0];
}

// theta_q(j) = clamp(atan2(s, c), 0, pi/2) for j < r_q, else 0
__global__ void theta_ragged_kernel(int N, int K, const double* __restrict__ cs,
                                    const int* __restrict__ rq, double* th) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)K * N) return;
  const int q = (int)(e / N), j = (int)(e % N);
  double t = 0.0;
  if (j < rq[q]) {
    t = atan2(cs[(2LL * q + 1) * N + j], cs[2LL * q * N + j]);
    t = fmin(fmax(t, 0.0), 1.5707963267948966);
  }
  th[e] = t;
}

// Remark (iv): theta_q(j) = clamp(pi/4 + asin(lambda_q(j) / sqrt(2)), 0, pi/2)
// for j < r_q, else 0
__global__ void theta_ragged_lambda_kernel(int N, int K, const double* __restrict__ lam,
                                           const int* __restrict__ rq, double* th) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)K * N) return;
  const int q = (int)(e / N), j = (int)(e % N);
  double t = 0.0;
  if (j < rq[q]) {
    const double x = fmin(fmax(lam[e], -1.0), 1.0);
    t = 0.7853981633974483 + asin(x * 0.7071067811865476);
    t = fmin(fmax(t, 0.0), 1.5707963267948966);
  }
  th[e] = t;
}

// dst(member q)(:, j) = src_q(0:n_q, perm_q[j]) for j < r_q, zero for r_q <= j < n_q
__global__ void ragged_gather_kernel(int N, const double* __restrict__ src, long long sstride,
                                     const int* __restrict__ nq, const int* __restrict__ rq,
                                     const long long* __restrict__ off, const int* __restrict__ perm,
                                     double* dst) {
  const int j = blockIdx.x, q = blockIdx.y;
  const int n = nq[q];
  if (j >= n) return;
  double* d = dst + off[q] + (long long)j * n;
  if (j < rq[q]) {
    const double* sc = src + (long long)q * sstride + (long long)perm[(long long)q * N + j] * N;
    for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = sc[i];
  } else {
    for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = 0.0;
  }
}

namespace {

dim3 grid_nn(long long NN, int nb) {
  long long g = (NN + 255) / 256;
  g = std::max<long long>(1, std::min<long long>(g, 1024));
  return dim3((unsigned)g, (unsigned)nb);
}

template <class T>
T* upload_vec(Arena& ar, const std::vector<T>& v, hipStream_t s) {
  T* d = static_cast<T*>(ar.alloc(std::max<size_t>(1, v.size()) * sizeof(T)));
  if (!v.empty()) h2d(d, v.data(), v.size() * sizeof(T), s);
  return d;
}

}  // namespace

// padded size of a problem of size n: the next multiple of step[0] up to 64
// (8 by default), of step[1] up to 256 (16), of step[2] beyond (64)
int batched_class_size(int n, const int step[3]) {
  const int st = n <= 64 ? step[0] : (n <= 256 ? step[1] : step[2]);
  return (n + st - 1) / st * st;
}

// the first W workers of the handle, each with its stream and second stream
// (created in this order, worker by worker)
void ensure_batch_workers(zcsd_handle* h, int W) {
  while ((int)h->workers.size() < W) {
    auto bw = std::make_unique<BatchWorker>();
    ZCSD_HIP(hipStreamCreateWithFlags(&bw->stream, hipStreamNonBlocking));
    ZCSD_HIP(hipStreamCreateWithFlags(&bw->aux, hipStreamNonBlocking));
    h->workers.push_back(std::move(bw));
  }
}

// arena bytes of one group of K problems of class size N: the iterates and
// products (216 N^2 doubles per problem), the Householder workspaces of the
// polars (2K problems, up to 8 terms each) and of Zolo-eig's sign functions
// (K blocks, up to 8 terms), and the Jacobi leaves (64 x 64 padded, at most
// N / 32 + 1 per problem).  For small N the fixed per-problem parts (32-wide
// panels, 64 x 64 leaves) outweigh the N^2 terms.
size_t batched_group_bytes(int N, size_t K) {
  const size_t NN = (size_t)N * N;
  const int k = (int)K;
  size_t b = K * (2 * 64 * NN + 64 * NN + 24 * NN) * sizeof(double);
  b += qr_work_bytes(QRShape::General, 2 * k, N, N, 32) +
       qr_work_bytes(QRShape::Stacked, 2 * k * ZOLO_RMAX, 2 * N, N, 32);
  if (N > 64)
    b += qr_work_bytes(QRShape::General, k, N, N, 32, N) +
         qr_work_bytes(QRShape::Stacked, k * ZOLO_RMAX, 2 * N, N, 32);
  const size_t leaves = K * (size_t)(N / 32 + 1);
  b += leaves * (2 * 64 * 64 + 2 * (size_t)N * 64 + 64) * sizeof(double);
  return b;
}

struct BatchedStats {
  int classes = 0, groups = 0, max_r = 0, eig_levels = 0, eig_splits = 0;
  int single = 0, repaired = 0;  // members sent to the single path; of those, repaired by Alg. 2
  double eig_offblock = 0.0, eig_coupling = 0.0;
  void merge(const BatchedStats& o) {
    groups += o.groups;
    max_r = std::max(max_r, o.max_r);
    eig_levels = std::max(eig_levels, o.eig_levels);
    eig_splits += o.eig_splits;
    eig_offblock = std::max(eig_offblock, o.eig_offblock);
    eig_coupling = std::max(eig_coupling, o.eig_coupling);
  }
};

// Size-class groups are independent, and each is a chain of dependent
// launches and host decisions that leaves much of the GPU idle for the small
// classes: up to this many run at once, each on its own host thread, stream
// and arena (the box's hardware queues per process: 4).

// One group: members of one size class with the same rank mode.  Returns
// false, having written nothing, when a full-rank group's shared lower bound
// l reached eps: a member may then have sigma_min(A_i) < eps, which the
// modified Zolo-pd leaves with a non-orthonormal W_i, and the batched kernels
// have no Algorithm 2 repair (Sec. 5.1); the caller runs those members
// through the single path, which has.
static bool csd_group(int N, const std::vector<int>& mem, bool deficient, const int* n_host,
                      const long long* off_host, const double* A1, const double* A2, double* U1,
                      double* U2, double* V1, std::vector<double>& theta_host,
                      const std::vector<long long>& toff, int* rank_host, const zcsd_opts& o,
                      BatchedStats& st, Arena& ar, hipStream_t s) {
  const int K = (int)mem.size();
  const long long NN = (long long)N * N;
  ArenaScope scope(ar);
  std::vector<int> nq(K);
  std::vector<long long> offq(K);
  for (int q = 0; q < K; ++q) {
    nq[q] = n_host[mem[q]];
    offq[q] = off_host[mem[q]];
  }
  int* d_n = upload_vec(ar, nq, s);
  long long* d_off = upload_vec(ar, offq, s);
  double* X = ar.dalloc((size_t)2 * K * NN);
  hipLaunchKernelGGL(pad_pack_kernel, grid_nn(NN, 2 * K), dim3(256), 0, s, N, A1, A2, d_off, d_n, X);
  ZCSD_CHECK_LAUNCH();
  // polars
  double* W = ar.dalloc((size_t)2 * K * NN);
  double* H = ar.dalloc((size_t)2 * K * NN);
  {
    ZoloPdArgs za;
    za.batch = 2 * K;
    za.n = N;
    za.alpha = 1.0;
    za.X = X; za.ldx = N; za.sx = NN;
    za.W = W; za.H = H;
    za.eps = o.eps; za.tol = o.tol;
    za.r_override = o.r_override;
    za.ell_override = o.ell_override;
    if (deficient) {
      if (za.ell_override <= 0.0) za.ell_override = o.eps;
      if (za.r_override <= 0) za.r_override = ZOLO_RMAX;
    }
    ZoloPdResult pr = zolo_pd_batched(za, ar, s);
    st.max_r = std::max(st.max_r, pr.r);
    if (!deficient && pr.ell <= o.eps * (1.0 + 1e-12)) return false;
  }
  // B
  const double mu = deficient ? o.mu : 0.0;
  double* B = ar.dalloc((size_t)K * NN);
  {
    double* G = nullptr;
    if (deficient) {
      G = ar.dalloc((size_t)K * NN);
      GemmBatch g;
      g.batch = K;
      g.transA = 1;
      g.m = N; g.n = N; g.k = N;
      g.A = X; g.lda = N; g.sA = 2 * NN;
      g.B = X; g.ldb = N; g.sB = 2 * NN;
      g.C = G; g.ldc = N; g.sC = NN;
      dgemm(g, s);
      g.A = X + NN; g.B = X + NN;
      g.beta = 1.0;
      dgemm(g, s);
    }
    hipLaunchKernelGGL(build_b_kernel, grid_nn(NN, K), dim3(256), 0, s, N, H, G, mu, d_n, B);
    ZCSD_CHECK_LAUNCH();
  }
  // eig
  double* V = ar.dalloc((size_t)K * NN);
  double* lam = ar.dalloc((size_t)K * N);
  {
    ZoloEigArgs ea;
    ea.n = N;
    ea.batch = K;
    ea.B = B; ea.ldb = N; ea.sB = NN;
    ea.lo = -1.0 - 1e-6;
    ea.hi = 3.0 + 1e-6;  // padding at 3, null space at mu < 3
    ea.V = V; ea.ldv = N; ea.sV = NN;
    ea.lam = lam; ea.sL = N;
    ea.n_leaf = o.n_leaf;
    ea.eps = o.eps; ea.tol = o.tol;
    // Alg. 3 keeps only the eigenpairs below (1 + mu)/2: the divide and
    // conquer splits first there and does not divide the part above it (the
    // null space at mu and the padding at 3).  Full rank keeps no bound: a
    // first split at 2 would be wasted on the problems without padding
    // (measured slower on the ragged batch)
    if (deficient) ea.keep_below = 0.5 * (1.0 + mu);
    ZoloEigResult er = zolo_eig(ea, ar, s);
    st.eig_levels = std::max(st.eig_levels, er.levels);
    st.eig_splits += er.splits;
    st.max_r = std::max(st.max_r, er.max_r);
    st.eig_offblock = std::max(st.eig_offblock, er.max_offblock);
    st.eig_coupling = std::max(st.eig_coupling, er.max_coupling);
  }
  // selection (ascending, so the kept pairs come first): lambda <= 2 keeps the
  // real spectrum [-1, 1] and drops the padding at 3; with the null space at mu
  // the threshold is (1 + mu) / 2 (Algorithm 3)
  const double keep_max = deficient ? 0.5 * (1.0 + mu) : 2.0;
  std::vector<double> lh((size_t)K * N);
  d2h(lh.data(), lam, lh.size() * sizeof(double), s);
  std::vector<int> rq(K);
  for (int q = 0; q < K; ++q) {
    int r = 0;
    while (r < N && lh[(size_t)q * N + r] <= keep_max) ++r;
    if (r > nq[q]) throw NumError(ZCSD_ENOCONV, "csd_batched: more real eigenpairs than columns");
    rq[q] = r;
    rank_host[mem[q]] = r;
  }
  int* d_r = upload_vec(ar, rq, s);
  // U_i = W_i V, T_i = H_i V (pairs of polars share V)
  double* Ut = ar.dalloc((size_t)2 * K * NN);
  double* T = ar.dalloc((size_t)2 * K * NN);
  {
    GemmBatch g;
    g.batch = K;
    g.batch2 = 2;
    g.m = N; g.n = N; g.k = N;
    g.A = W; g.lda = N; g.sA = 2 * NN; g.sA2 = NN;
    g.B = V; g.ldb = N; g.sB = NN; g.sB2 = 0;
    g.C = Ut; g.ldc = N; g.sC = 2 * NN; g.sC2 = NN;
    dgemm(g, s);
    if (deficient) {
      // the Newton-Schulz correction of the single path on the kept columns:
      // masking the others to zero makes the full products act on them alone
      hipLaunchKernelGGL(mask_cols_kernel, grid_nn(NN, 2 * K), dim3(256), 0, s, N, Ut, d_r);
      ZCSD_CHECK_LAUNCH();
      double* Gr = T;
      double* Tc = ar.dalloc((size_t)2 * K * NN);
      for (int it = 0; it < 2; ++it) {
        GemmBatch q;
        q.batch = 2 * K;
        q.transA = 1;
        q.m = N; q.n = N; q.k = N;
        q.A = Ut; q.lda = N; q.sA = NN;
        q.B = Ut; q.ldb = N; q.sB = NN;
        q.C = Gr; q.ldc = N; q.sC = NN;
        dgemm(q, s);
        GemmBatch u = q;
        u.transA = 0;
        u.A = Ut; u.B = Gr; u.C = Tc;
        dgemm(u, s);
        const long long tot = 2LL * K * NN;  // Ut = 1.5 Ut - 0.5 Tc
        hipLaunchKernelGGL(axpby_flat_kernel, dim3((unsigned)std::min<long long>((tot + 255) / 256, 4096)),
                           dim3(256), 0, s, tot, -0.5, Tc, 1.5, Ut);
        ZCSD_CHECK_LAUNCH();
      }
    }
    if (o.postprocess != 2) {
      g.A = H;
      g.C = T;
      dgemm(g, s);
    }
  }
  double* th = ar.dalloc((size_t)K * N);
  const long long tot = (long long)K * N;
  if (o.postprocess == 2) {
    hipLaunchKernelGGL(theta_ragged_lambda_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                       s, N, K, lam, d_r, th);
    ZCSD_CHECK_LAUNCH();
  } else {
    double* cs = ar.dalloc((size_t)2 * K * N);
    hipLaunchKernelGGL(coldot_ragged_kernel, dim3(N, 2 * K), dim3(64), 0, s, N, V, T, d_n, cs);
    ZCSD_CHECK_LAUNCH();
    hipLaunchKernelGGL(theta_ragged_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, N,
                       K, cs, d_r, th);
    ZCSD_CHECK_LAUNCH();
  }
  // order by ascending theta per problem, gather into the packed outputs
  std::vector<double> thh((size_t)K * N);
  d2h(thh.data(), th, thh.size() * sizeof(double), s);
  std::vector<int> perm((size_t)K * N);
  for (int q = 0; q < K; ++q) {
    int* pq = perm.data() + (size_t)q * N;
    std::iota(pq, pq + N, 0);
    const double* tq = thh.data() + (size_t)q * N;
    std::stable_sort(pq, pq + rq[q], [&](int x, int y) { return tq[x] < tq[y]; });
    double* out = theta_host.data() + toff[mem[q]];
    for (int j = 0; j < nq[q]; ++j) out[j] = (j < rq[q]) ? tq[pq[j]] : 0.0;
  }
  int* d_perm = upload_vec(ar, perm, s);
  hipLaunchKernelGGL(ragged_gather_kernel, dim3(N, K), dim3(64), 0, s, N, Ut, 2 * NN, d_n, d_r,
                     d_off, d_perm, U1);
  ZCSD_CHECK_LAUNCH();
  hipLaunchKernelGGL(ragged_gather_kernel, dim3(N, K), dim3(64), 0, s, N, Ut + NN, 2 * NN, d_n,
                     d_r, d_off, d_perm, U2);
  ZCSD_CHECK_LAUNCH();
  hipLaunchKernelGGL(ragged_gather_kernel, dim3(N, K), dim3(64), 0, s, N, V, NN, d_n, d_r, d_off,
                     d_perm, V1);
  ZCSD_CHECK_LAUNCH();
  HostSync::sync(s);
  return true;
}

}  // namespace zcsd

using namespace zcsd;

extern "C" zcsd_status zcsd_dcsd_batched(zcsd_handle* handle, int batch, const int* n_host,
                                         const long long* off_host, const double* d_A1,
                                         const double* d_A2, double* d_U1, double* d_U2,
                                         double* d_V1, double* d_theta, int* rank_host,
                                         const zcsd_opts* opts, zcsd_info* info) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(batch >= 1 && batch <= 65535, "csd_batched: 1 <= batch <= 65535");
    ZCSD_REQUIRE(n_host && off_host && rank_host, "csd_batched: NULL host array");
    ZCSD_REQUIRE(d_A1 && d_A2 && d_U1 && d_U2 && d_V1 && d_theta, "csd_batched: NULL pointer");
    zcsd_opts o;
    zcsd_default_opts(&o);
    if (opts) o = *opts;
    ZCSD_REQUIRE(o.r_override >= 0 && o.r_override <= ZOLO_RMAX, "csd_batched: r_override out of range");
    ZCSD_REQUIRE(o.prec == ZCSD_FP64, "csd_batched: FP64 only");
    ZCSD_REQUIRE(o.eps > 0.0 && o.eps < 1.0 && o.tol > 0.0, "csd_batched: eps/tol out of range");
    ZCSD_REQUIRE(o.mu > 1.0 && o.mu < 3.0, "csd_batched: mu must lie in (1, 3)");
    ZCSD_REQUIRE(o.postprocess >= 0 && o.postprocess <= 2, "csd_batched: postprocess must be 0, 1 or 2");
    std::vector<long long> toff(batch + 1, 0);
    for (int k = 0; k < batch; ++k) {
      ZCSD_REQUIRE(n_host[k] >= 1 && n_host[k] <= 4096, "csd_batched: sizes must lie in [1, 4096]");
      ZCSD_REQUIRE(off_host[k] >= 0, "csd_batched: negative offset");
      toff[k + 1] = toff[k] + n_host[k];
    }
    ZCSD_HIP(hipSetDevice(handle->device));
    hipStream_t s = handle->stream;
    Arena& ar = handle->arena;
    ar.reset();
    // workspace ceiling per chunk (each of the concurrent workers holds one)
    const int n_workers = std::max(1, handle->tune_workers);
    const size_t cap_bytes = ((size_t)48 << 30) / n_workers;
    // members per chunk: the workspace ceiling, and the launch grids of the
    // polars, whose second dimension (<= 65535) enumerates 2 polars x r <= 8
    // terms per member
    auto chunk_of = [&](int N, size_t members) {
      size_t c = std::min<size_t>(members, 65535 / (2 * ZOLO_RMAX));
      while (c > 1 && batched_group_bytes(N, c) > cap_bytes) c = (c + 1) / 2;
      return std::max<size_t>(1, c);
    };
    // small full-rank problems: whole CSDs of one workgroup each, one
    // persistent launch beside the class groups (candidates by size here, by
    // rank below); not when the options fix l or r, or split blocks <= 64
    int tier_max[8], tier_per_cu[8];
    const int n_tiers = small_csd_tiers(tier_max, tier_per_cu);
    const int small_lim = (o.r_override == 0 && o.ell_override <= 0.0)
                              ? std::min(std::min(handle->tune_small_max, tier_max[0]), o.n_leaf)
                              : 0;
    // the tier of a size: the last (smallest) tier that holds it
    auto tier_of = [&](int n) {
      int t = 0;
      while (t + 1 < n_tiers && n <= tier_max[t + 1]) ++t;
      return t;
    };
    int n_cand = 0, tier_cand[8] = {0};
    for (int k = 0; k < batch; ++k)
      if (n_host[k] <= small_lim) {
        ++n_cand;
        ++tier_cand[tier_of(n_host[k])];
      }
    int n_cu = 1;
    ZCSD_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, handle->device));
    // grids: as many workgroups as fit on the device at once (per tier)
    int grid_max[8];
    for (int t = 0; t < n_tiers; ++t) grid_max[t] = std::min(tier_cand[t], tier_per_cu[t] * n_cu);
    const size_t small_bytes =
        n_cand ? small_csd_scratch_bytes(grid_max) + (size_t)batch * 64 + ((size_t)1 << 20) : 0;
    ar.reserve(((size_t)64 << 20) + (size_t)batch * 64 + small_bytes);
    // ranks (Remark (vi)) for every problem
    std::vector<double> ss((size_t)2 * batch);
    {
      ArenaScope sc(ar);
      std::vector<int> nv(n_host, n_host + batch);
      std::vector<long long> ov(off_host, off_host + batch);
      int* d_n = upload_vec(ar, nv, s);
      long long* d_off = upload_vec(ar, ov, s);
      double* d_ss = ar.dalloc((size_t)2 * batch);
      hipLaunchKernelGGL(ragged_sumsq_kernel, dim3(batch, 2), dim3(256), 0, s, d_A1, d_A2, d_off, d_n,
                         d_ss);
      ZCSD_CHECK_LAUNCH();
      d2h(ss.data(), d_ss, ss.size() * sizeof(double), s);
    }
    std::vector<char> deficient(batch, 0);
    for (int k = 0; k < batch; ++k) {
      const double f2 = ss[2 * k] + ss[2 * k + 1];
      if (!std::isfinite(f2)) throw ArgError("csd_batched: input contains NaN or Inf");
      const long long rA = std::llround(f2);
      if (o.rank_mode == ZCSD_RANK_FULL) deficient[k] = 0;
      else if (o.rank_mode == ZCSD_RANK_DEFICIENT) deficient[k] = 1;
      else {
        if (std::fabs(f2 - (double)rA) > 0.25)
          throw NumError(ZCSD_ENOTISO, "csd_batched: ||A||_F^2 is not close to an integer rank");
        deficient[k] = rA < n_host[k];
      }
    }
    std::vector<int> small;
    std::vector<char> is_small(batch, 0);
    for (int k = 0; k < batch; ++k)
      if (!deficient[k] && n_host[k] <= small_lim) {
        small.push_back(k);
        is_small[k] = 1;
      }
    // largest first: the workgroups take the list in turn
    std::stable_sort(small.begin(), small.end(), [&](int x, int y) { return n_host[x] > n_host[y]; });
    // classes of the other problems
    std::map<int, std::vector<int>> cls;
    for (int k = 0; k < batch; ++k)
      if (!is_small[k]) cls[batched_class_size(n_host[k], handle->tune_step)].push_back(k);
    std::vector<double> theta_host(toff[batch], 0.0);
    BatchedStats st;
    st.classes = (int)cls.size();
    // groups (members of one class with one rank mode, in chunks), costed by
    // their flops plus a fixed latency of about 200 class-64 problems
    struct Grp {
      int N;
      bool def;
      std::vector<int> mem;
      double cost;
    };
    std::vector<Grp> groups;
    for (auto& kv : cls) {
      const int N = kv.first;
      const size_t chunk = chunk_of(N, kv.second.size());
      for (int def = 0; def < 2; ++def) {
        std::vector<int> grp;
        for (int k : kv.second)
          if ((int)deficient[k] == def) grp.push_back(k);
        for (size_t c0 = 0; c0 < grp.size(); c0 += chunk) {
          Grp g;
          g.N = N;
          g.def = def != 0;
          g.mem.assign(grp.begin() + c0, grp.begin() + std::min(grp.size(), c0 + chunk));
          g.cost = (double)g.mem.size() * N * N * N + 200.0 * 64 * 64 * 64;
          groups.push_back(std::move(g));
        }
      }
    }
    // largest cost first onto the least loaded worker
    const int W = std::max(1, std::min<int>(n_workers, (int)groups.size()));
    std::vector<int> order(groups.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return groups[x].cost > groups[y].cost; });
    std::vector<std::vector<int>> assign(W);
    std::vector<double> load(W, 0.0);
    for (int gi : order) {
      const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      assign[w].push_back(gi);
      load[w] += groups[gi].cost;
    }
    ensure_batch_workers(handle, W);
    // the workers start after everything queued on the caller's stream
    hipEvent_t ready = nullptr;
    ZCSD_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    ZCSD_HIP(hipEventRecord(ready, s));
    int* d_small_status = nullptr;
    if (!small.empty()) {
      int tier_count[8] = {0}, grid[8] = {0};
      for (int k : small) ++tier_count[tier_of(n_host[k])];
      for (int t = 0; t < n_tiers; ++t) grid[t] = std::min(tier_count[t], grid_max[t]);
      std::vector<int> nv(n_host, n_host + batch);
      std::vector<long long> ov(off_host, off_host + batch), tv(toff.begin(), toff.begin() + batch);
      int* d_list = upload_vec(ar, small, s);
      int* d_nv = upload_vec(ar, nv, s);
      long long* d_ov = upload_vec(ar, ov, s);
      long long* d_tv = upload_vec(ar, tv, s);
      d_small_status = ar.ialloc(small.size());
      double* scratch = ar.dalloc(small_csd_scratch_bytes(grid) / sizeof(double));
      small_csd_launch(tier_count, d_list, d_nv, d_ov, d_tv, d_A1, d_A2, d_U1, d_U2, d_V1, d_theta, o.eps,
                       o.tol, o.postprocess == 2, grid, scratch, d_small_status, ar, s);
    }
    const int dev = handle->device;
    std::vector<BatchedStats> wst(W);
    std::vector<std::vector<int>> wsingle(W);
    std::vector<std::exception_ptr> werr(W);
    auto work = [&](int w) {
      try {
        ZCSD_HIP(hipSetDevice(dev));
        BatchWorker& bw = *handle->workers[w];
        set_thread_aux_stream(bw.aux);
        GemmTileScope tile_scope(handle->tune_tile128_min);
        size_t need_w = 0;
        for (int gi : assign[w]) need_w = std::max(need_w, batched_group_bytes(groups[gi].N, groups[gi].mem.size()));
        bw.arena.reset();
        bw.arena.reserve(need_w + ((size_t)256 << 20));
        ZCSD_HIP(hipStreamWaitEvent(bw.stream, ready, 0));
        for (int gi : assign[w]) {
          const Grp& g = groups[gi];
          ++wst[w].groups;
          if (!csd_group(g.N, g.mem, g.def, n_host, off_host, d_A1, d_A2, d_U1, d_U2, d_V1,
                         theta_host, toff, rank_host, o, wst[w], bw.arena, bw.stream))
            wsingle[w].insert(wsingle[w].end(), g.mem.begin(), g.mem.end());
        }
        ZCSD_HIP(hipStreamSynchronize(bw.stream));
        set_thread_aux_stream(nullptr);
      } catch (...) {
        set_thread_aux_stream(nullptr);
        werr[w] = std::current_exception();
      }
    };
    if (W == 1) {
      work(0);
    } else {
      std::vector<std::thread> th;
      for (int w = 1; w < W; ++w) th.emplace_back(work, w);
      work(0);
      for (auto& t : th) t.join();
    }
    (void)hipEventDestroy(ready);
    for (int w = 0; w < W; ++w)
      if (werr[w]) std::rethrow_exception(werr[w]);
    std::vector<int> single;  // members of full-rank groups whose l reached eps
    for (int w = 0; w < W; ++w) {
      st.merge(wst[w]);
      single.insert(single.end(), wsingle[w].begin(), wsingle[w].end());
    }
    if (!small.empty()) {
      // the one-workgroup CSDs: their angles are in d_theta (no class group
      // writes there); problems whose l reached eps go to the single path
      std::vector<int> sst(small.size());
      d2h(sst.data(), d_small_status, sst.size() * sizeof(int), s);
      std::vector<double> thd(toff[batch]);
      d2h(thd.data(), d_theta, thd.size() * sizeof(double), s);
      for (size_t i = 0; i < small.size(); ++i) {
        const int k = small[i];
        if ((sst[i] & 255) == 0) {
          rank_host[k] = n_host[k];
          std::copy(thd.begin() + toff[k], thd.begin() + toff[k + 1], theta_host.begin() + toff[k]);
          st.max_r = std::max(st.max_r, sst[i] >> 8);
        } else {
          single.push_back(k);
        }
      }
    }
    std::sort(single.begin(), single.end());
    // the single path (with Algorithm 2) for those members, one at a time;
    // no arena allocation is live between groups, so the arena may grow here
    for (int k : single) {
      const int n = n_host[k];
      ar.reset();
      ar.reserve(csd_workspace_bytes(n) + ((size_t)64 << 20));
      double* th = ar.dalloc(n);
      zcsd_opts o1 = o;
      o1.rank_mode = ZCSD_RANK_FULL;
      bool rep = false;
      rank_host[k] = csd_single_member(n, d_A1 + off_host[k], d_A2 + off_host[k], d_U1 + off_host[k],
                                       d_U2 + off_host[k], d_V1 + off_host[k], th, o1, ar, s, &rep);
      d2h(theta_host.data() + toff[k], th, n * sizeof(double), s);
      ++st.single;
      st.repaired += rep ? 1 : 0;
    }
    h2d(d_theta, theta_host.data(), theta_host.size() * sizeof(double), s);
    ZCSD_HIP(hipStreamSynchronize(s));
    if (info) {
      *info = zcsd_info{};
      info->rank = batch;
      info->r_used[0] = info->r_used[1] = st.max_r;
      info->eig_levels = st.eig_levels;
      info->eig_splits = st.eig_splits;
      info->eig_offblock = st.eig_offblock;
      info->eig_coupling = st.eig_coupling;
      info->repair = st.repaired;
    }
  });
}
