// Zolo-eig (Sec. 5): symmetric eigendecomposition by spectral divide and
// conquer on the matrix sign function, which is the polar factor of B - sI.
//
// Level by level, every unfinished block B_b (size n_b, spectrum inside
// [lo_b, hi_b]) is processed in one batch, zero-padded to the level's largest
// size N with the padding decoupled from the real part:
//   1. shift s_b (median of diag B_b, kept inside (lo_b, hi_b)); alpha_b =
//      max(hi_b - s_b, s_b - lo_b) bounds ||B_b - s_b I||_2; X_b = (B_b - s_b I)/alpha_b
//      with 1 on the padded diagonal;
//   2. W_b = sign(X_b) by batched Zolo-pd; P_b = (W_b + W_b^T)/4 + I/2 is the
//      spectral projector onto the eigenvalues above s_b (plus the padding);
//      n+_b = round(trace P_b over the real part);
//   3. [V+ V-] = Q of the Householder QR of P_b Omega_b (Omega random on the
//      real part, identity on the padding, so Q = diag(Q_real, I) exactly),
//      refined by one step of subspace iteration on P_b (first-order form);
//   4. B'_b = Q^T B_b Q, V_b <- V_b Q; the diagonal blocks of B'_b of sizes
//      n+ and n_b - n+ are the children, with spectra in [s_b, hi_b] and
//      [lo_b, s_b]; ||B'_21||_F / ||B||_F is recorded.
// A split with n+ in {0, n_b} only moves the interval (bisection on s).
// Before each split the interval is tightened to mean_b -+ ||B_b - mean_b I||_F,
// which holds every eigenvalue of the block.
// Blocks of at most n_leaf go to batched Jacobi, all of them in one launch
// after the last level (a leaf is independent of the rest, and the Jacobi
// launch is latency-bound: one launch of a few hundred leaves costs about as
// much as one of a few); blocks whose spread
// ||B_b - mean I||_F is below 4 u max(|lo|, |hi|) are already diagonal to
// working accuracy and are finished as they are.  Eigenpairs are finally sorted.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <numeric>
#include <vector>

#include "zcsd_api_guard.h"
#include "zcsd_eig.h"
#include "zcsd_internal.h"
#include "zcsd_la.h"
#include "zcsd_zolo.h"

namespace zcsd {

// ---------------------------------------------------------------------------
// kernels

__global__ void copy_blocks_kernel(const double* __restrict__ src, double* dst,
                                   const CopyDesc* __restrict__ d) {
  const CopyDesc c = d[blockIdx.y];
  const long long total = (long long)c.rows * c.cols;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % c.rows), j = (int)(e / c.rows);
    dst[c.dst_off + i + (long long)j * c.dst_ld] = src[c.src_off + i + (long long)j * c.src_ld];
  }
}

// X_b = (B_b - s_b I) * inva_b on the real n_b x n_b part, identity on the padding
__global__ void form_shifted_kernel(int N, const double* __restrict__ Bp, double* X,
                                    const int* __restrict__ nb, const double* __restrict__ sh,
                                    const double* __restrict__ inva) {
  const long long b = blockIdx.y;
  const long long NN = (long long)N * N;
  const int m = nb[b];
  const double s = sh[b], f = inva[b];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < NN;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % N), j = (int)(e / N);
    double v;
    if (i < m && j < m) v = (Bp[b * NN + e] - (i == j ? s : 0.0)) * f;
    else v = (i == j) ? 1.0 : 0.0;
    X[b * NN + e] = v;
  }
}

// P_b = (W_b + W_b^T)/4 + I/2 in place on the real n_b x n_b part; the padding
// is reset to exactly I and its coupling to the real part to exactly 0.  Zolo-pd
// keeps that coupling at rounding level only (the tall-panel QR does not
// preserve exact zeros), and the QR of the rank-deficient P Omega would turn
// rounding-level coupling into O(1) coupling on its trailing (null) columns.
__global__ void projector_kernel(int N, double* W, const int* __restrict__ nb) {
  const long long b = blockIdx.y;
  const long long NN = (long long)N * N;
  const int m = nb[b];
  double* Wb = W + b * NN;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < NN;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % N), j = (int)(e / N);
    if (i >= m || j >= m) {
      Wb[e] = (i == j) ? 1.0 : 0.0;
    } else if (i > j) {
      const double v = 0.25 * (Wb[e] + Wb[j + (long long)i * N]);
      Wb[e] = v;
      Wb[j + (long long)i * N] = v;
    } else if (i == j) {
      Wb[e] = 0.5 * Wb[e] + 0.5;
    }
  }
}

__global__ void trace_real_kernel(int N, const double* __restrict__ P, const int* __restrict__ nb,
                                  double* tr) {
  const long long b = blockIdx.x;
  const int m = nb[b];
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) acc += P[b * (long long)N * N + i + (long long)i * N];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) tr[b] = red[0];
}

// Omega_b: uniform(-1, 1) on the real part (counter hash), identity on the padding
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__global__ void omega_kernel(int N, double* Om, const int* __restrict__ nb,
                             unsigned long long seed) {
  const long long b = blockIdx.y;
  const long long NN = (long long)N * N;
  const int m = nb[b];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < NN;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % N), j = (int)(e / N);
    double v;
    if (i < m && j < m) {
      const unsigned long long h = mix64(seed ^ mix64(((unsigned long long)i << 32) | (unsigned)j));
      v = 2.0 * ((double)(h >> 11) * 0x1.0p-53) - 1.0;
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
    Om[b * NN + e] = v;
  }
}

// out[b] = ||B_b - d_b I||_F^2 over the n_b x n_b real part (diag shift d_b)
// K_b = [0 -X^T; X 0] on the real n_b x n_b part (X = Z_b(np:n_b, 0:np)), zero
// elsewhere; the upper block is built from the lower one, so K is exactly skew.
__global__ void coupling_skew_kernel(int N, const double* __restrict__ Z, double* K,
                                     const int* __restrict__ nb, const int* __restrict__ npos) {
  const long long b = blockIdx.y;
  const long long NN = (long long)N * N;
  const int m = nb[b], p = npos[b];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < NN;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % N), j = (int)(e / N);
    double v = 0.0;
    if (i < m && j < m) {
      if (i >= p && j < p) v = Z[b * NN + e];
      else if (i < p && j >= p) v = -Z[b * NN + j + (long long)i * N];
    }
    K[b * NN + e] = v;
  }
}

// E_b -= Bq_b on the real n_b x n_b part; zero elsewhere
__global__ void sub_real_kernel(int N, double* E, const double* __restrict__ Bq,
                                const int* __restrict__ nb) {
  const long long b = blockIdx.y;
  const long long NN = (long long)N * N;
  const int m = nb[b];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < NN;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % N), j = (int)(e / N);
    E[b * NN + e] = (i < m && j < m) ? E[b * NN + e] - Bq[b * NN + e] : 0.0;
  }
}

__global__ void diag_kernel(int N, const double* __restrict__ Bp, const int* __restrict__ nb,
                            double* out) {
  const long long b = blockIdx.y;
  const int m = nb[b];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    out[b * (long long)N + i] = Bp[b * (long long)N * N + i + (long long)i * N];
}

// out[b] = max |X_b(i, j)| over pairs with exactly one of i, j in the padding
__global__ void offpad_kernel(int N, const double* __restrict__ X, const int* __restrict__ nb,
                              double* out) {
  const long long b = blockIdx.x;
  const int m = nb[b];
  double mx = 0.0;
  for (long long e = threadIdx.x; e < (long long)N * N; e += blockDim.x) {
    const int i = (int)(e % N), j = (int)(e / N);
    if ((i < m) != (j < m)) mx = fmax(mx, fabs(X[b * (long long)N * N + e]));
  }
  __shared__ double red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = red[0];
}

static dim3 grid2(long long total, int batch) {
  long long g = (total + 255) / 256;
  g = std::max<long long>(1, std::min<long long>(g, 1024));
  return dim3((unsigned)g, (unsigned)batch);
}

void copy_blocks(const double* src, double* dst, const std::vector<CopyDesc>& d, Arena& ar,
                 hipStream_t s) {
  if (d.empty()) return;
  ArenaScope sc(ar);
  CopyDesc* dd = static_cast<CopyDesc*>(ar.alloc(d.size() * sizeof(CopyDesc)));
  h2d(dd, d.data(), d.size() * sizeof(CopyDesc), s);
  long long mx = 1;
  for (const auto& c : d) mx = std::max<long long>(mx, (long long)c.rows * c.cols);
  for (size_t o = 0; o < d.size(); o += 65535) {
    const unsigned cnt = (unsigned)std::min<size_t>(65535, d.size() - o);
    hipLaunchKernelGGL(copy_blocks_kernel, grid2(mx, cnt), dim3(256), 0, s, src, dst, dd + o);
    ZCSD_CHECK_LAUNCH();
  }
}

// ---------------------------------------------------------------------------
// host driver

namespace {
struct Blk {
  int n;
  int prob = 0;  // which problem of the batch
  double lo, hi;
  // location at the current level
  const double* B;  // n x n, ld ldB
  long long ldB;
  const double* V;  // nglob x n, ld nglob
  int tries = 0;
  double split_at = 0.0;  // with has_split_at: the shift of this block's split
  bool has_split_at = false;
  bool drop = false;      // eigenpairs not wanted: finished as a scalar block
};

template <class T>
T* upload(Arena& ar, const std::vector<T>& v, hipStream_t s) {
  T* d = static_cast<T*>(ar.alloc(std::max<size_t>(1, v.size()) * sizeof(T)));
  if (!v.empty()) h2d(d, v.data(), v.size() * sizeof(T), s);
  return d;
}
}  // namespace

// ZCSD_EIG_TIMES=1: one line per level with its blocks, Zolotarev degree and
// wall times (the stream is drained at the level's start, around the sign
// function and at its end; nothing else changes)
static bool level_times_enabled() {
  static const bool v = [] {
    const char* e = std::getenv("ZCSD_EIG_TIMES");
    return e && e[0] && e[0] != '0';
  }();
  return v;
}

static double wall_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

ZoloEigResult zolo_eig(const ZoloEigArgs& a, Arena& ar, hipStream_t s) {
  const int n = a.n;
  const int nprob = a.batch;
  ZoloEigResult res;
  ZCSD_REQUIRE(n >= 1 && nprob >= 1, "zolo_eig: n >= 1, batch >= 1");
  const int nleaf = std::max(1, std::min(a.n_leaf, 64));
  const long long nn = (long long)n * n;
  ArenaScope scope(ar);
  // mixed mode: every product of the divide and conquer runs on the FP32 matrix
  // cores (the compact-WY factors of its QRs excepted); the caller
  // re-orthogonalises the basis in FP64
  GemmLowpScope lowp_scope(a.lowp);

  // Frobenius norm of B (largest over the batch; for the off-block ratio)
  double bnorm2 = 0.0;
  {
    double* d_ss = ar.dalloc(nprob);
    sumsq(nprob, n, n, a.B, a.ldb, a.sB, d_ss, ar, s);
    std::vector<double> ss(nprob);
    d2h(ss.data(), d_ss, nprob * sizeof(double), s);
    for (double v : ss) bnorm2 = std::max(bnorm2, v);
  }
  const double bnorm = std::sqrt(bnorm2);
  // A block is finished without splitting only when ||B_blk - mean I||_F (an upper
  // bound of its 2-norm) is a few units of roundoff of ||B||_2 <= max(|lo|, |hi|):
  // then any orthonormal basis of it is an eigenbasis to working accuracy.
  const double bmax = std::max(std::fabs(a.lo), std::fabs(a.hi));
  const double scalar_tol = 4.0 * 0x1p-53 * std::max(bmax, 1e-300);

  // output assembly: unsorted eigenvectors/values per problem
  double* Vout = ar.dalloc((size_t)nprob * nn);
  std::vector<std::vector<double>> lam_out(nprob);
  std::vector<int> col_out(nprob, 0);

  // level 0: every problem whole, V = I
  double* V0 = ar.dalloc((size_t)nprob * nn);
  set_identity(nprob, n, n, 1.0, V0, n, nn, s);
  std::vector<Blk> active;
  for (int p = 0; p < nprob; ++p) {
    Blk r;
    r.n = n;
    r.prob = p;
    r.lo = a.lo;
    r.hi = a.hi;
    r.B = a.B + (long long)p * a.sB;
    r.ldB = a.ldb;
    r.V = V0 + (long long)p * nn;
    if (a.keep_below < a.hi) {
      // only the eigenpairs below keep_below are wanted: the first split is
      // there and the part above is not divided further
      r.split_at = a.keep_below;
      r.has_split_at = true;
    }
    active.push_back(r);
  }
  unsigned long long seed = 0x5DEECE66DULL;

  // blocks parked for the end: leaves (their matrix block, ld ldB, and their
  // n x nb basis, ld n, in the buffers of the level that produced them)
  struct Parked {
    const double* B;
    int ldB;
    const double* V;
    int nb, prob;
  };
  std::vector<Parked> parked;
  std::vector<long long> parked_cols(nprob, 0);
  // leaves: Jacobi on 64 x 64 padded copies, then V_b Q_leaf into the output
  auto solve_leaves = [&]() {
    if (parked.empty()) return;
    {
      const int nl = (int)parked.size();
      const int L = 64;
      double* Lb = ar.dalloc((size_t)nl * L * L);
      double* Lv = ar.dalloc((size_t)nl * L * L);
      double* Ll = ar.dalloc((size_t)nl * L);
      double* LV = ar.dalloc((size_t)nl * n * L);
      set_identity(nl, L, L, 0.0, Lv, L, (long long)L * L, s);
      set_identity(nl, n, L, 0.0, LV, n, (long long)n * L, s);
      // the parked blocks come from several levels' buffers: offsets from the
      // lowest address (one flat device address space), two copy launches
      const double* bbase = parked[0].B;
      const double* vbase = parked[0].V;
      for (const Parked& pk : parked) {
        bbase = std::min(bbase, pk.B);
        vbase = std::min(vbase, pk.V);
      }
      std::vector<CopyDesc> cb, cv;
      std::vector<int> szs;
      for (int q = 0; q < nl; ++q) {
        const Parked& pk = parked[q];
        cb.push_back({(long long)(pk.B - bbase), (long long)q * L * L, pk.ldB, L, pk.nb, pk.nb});
        cv.push_back({(long long)(pk.V - vbase), (long long)q * n * L, n, n, n, pk.nb});
        szs.push_back(pk.nb);
      }
      copy_blocks(bbase, Lb, cb, ar, s);
      copy_blocks(vbase, LV, cv, ar, s);
      int* d_sz = upload(ar, szs, s);
      jacobi_batched(nl, d_sz, Lb, L, (long long)L * L, Lv, L, (long long)L * L, Ll, s);
      double* LVo = ar.dalloc((size_t)nl * n * L);
      GemmBatch g;
      g.batch = nl;
      g.m = n; g.n = L; g.k = L;
      g.A = LV; g.lda = n; g.sA = (long long)n * L;
      g.B = Lv; g.ldb = L; g.sB = (long long)L * L;
      g.C = LVo; g.ldc = n; g.sC = (long long)n * L;
      dgemm(g, s);
      std::vector<double> ll((size_t)nl * L);
      d2h(ll.data(), Ll, ll.size() * sizeof(double), s);
      if (log_enabled() && nprob == 1) {
        // leaf invariants: ||LVo^T B LVo - diag(lam)||_F per leaf, ||LVo^T LVo - I||_F
        ArenaScope ds(ar);
        double* BV = ar.dalloc((size_t)nl * n * L);
        double* E = ar.dalloc((size_t)nl * L * L);
        double* E2 = ar.dalloc((size_t)nl * L * L);
        GemmBatch g1;
        g1.batch = nl;
        g1.m = n; g1.n = L; g1.k = n;
        g1.A = a.B; g1.lda = a.ldb; g1.sA = 0;
        g1.B = LVo; g1.ldb = n; g1.sB = (long long)n * L;
        g1.C = BV; g1.ldc = n; g1.sC = (long long)n * L;
        dgemm(g1, s);
        GemmBatch g2;
        g2.batch = nl;
        g2.transA = 1;
        g2.m = L; g2.n = L; g2.k = n;
        g2.A = LVo; g2.lda = n; g2.sA = (long long)n * L;
        g2.B = BV; g2.ldb = n; g2.sB = (long long)n * L;
        g2.C = E; g2.ldc = L; g2.sC = (long long)L * L;
        dgemm(g2, s);
        g2.B = LVo;
        g2.C = E2;
        dgemm(g2, s);
        std::vector<double> eh((size_t)nl * L * L), e2h((size_t)nl * L * L);
        d2h(eh.data(), E, eh.size() * sizeof(double), s);
        d2h(e2h.data(), E2, e2h.size() * sizeof(double), s);
        for (int q = 0; q < nl; ++q) {
          const int m = szs[q];
          double r1 = 0.0, r2 = 0.0;
          for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) {
              const double v = eh[(size_t)q * L * L + i + j * L] - (i == j ? ll[(size_t)q * L + i] : 0.0);
              const double w2 = e2h[(size_t)q * L * L + i + j * L] - (i == j ? 1.0 : 0.0);
              r1 += v * v;
              r2 += w2 * w2;
            }
          std::fprintf(stderr, "[zcsd] eig level %d leaf %d n=%d ||VtBV-L||=%.2e ||VtV-I||=%.2e\n",
                       res.levels, q, m, std::sqrt(r1), std::sqrt(r2));
        }
      }
      std::vector<CopyDesc> co;
      for (int q = 0; q < nl; ++q) {
        const Parked& pk = parked[q];
        const int p = pk.prob;
        co.push_back({(long long)q * n * L, p * nn + (long long)col_out[p] * n, n, n, n, pk.nb});
        for (int i = 0; i < pk.nb; ++i) lam_out[p].push_back(ll[(size_t)q * L + i]);
        col_out[p] += pk.nb;
      }
      copy_blocks(LVo, Vout, co, ar, s);
    }
    parked.clear();
  };
  const bool lt = level_times_enabled();
  double lt_start = 0.0, lt_sign = 0.0;
  int lt_r = 0, lt_ns = 0, lt_N = 0, lt_blocks = 0;
  while (!active.empty()) {
    ++res.levels;
    if (lt) {
      HostSync::sync(s);
      lt_start = wall_ms();
      lt_sign = 0.0;
      lt_r = lt_ns = lt_N = 0;
      lt_blocks = (int)active.size();
    }
    // --- classify: leaves / scalar / split --------------------------------
    std::vector<Blk> leaves, split;
    for (auto& b : active) {
      if (b.n <= nleaf) leaves.push_back(b);
      else split.push_back(b);
    }
    // pack every block of this level into padded arrays
    std::vector<Blk> all = split;
    all.insert(all.end(), leaves.begin(), leaves.end());
    const int nblk = (int)all.size();
    int N = 1;
    for (auto& b : all) N = std::max(N, b.n);
    const long long NN = (long long)N * N;
    double* Bp = ar.dalloc((size_t)nblk * NN);
    double* Vp = ar.dalloc((size_t)nblk * n * N);
    set_identity(nblk, N, N, 0.0, Bp, N, NN, s);
    set_identity(nblk, n, N, 0.0, Vp, n, (long long)n * N, s);
    {
      // the blocks of a level come from different buffers (the input, children of
      // splits, re-tried blocks): offsets are taken from the lowest block address
      // (one flat device address space), so each level is two copy launches
      const double* bbase = all[0].B;
      const double* vbase = all[0].V;
      for (int k = 1; k < nblk; ++k) {
        bbase = std::min(bbase, all[k].B);
        vbase = std::min(vbase, all[k].V);
      }
      std::vector<CopyDesc> cb, cv;
      for (int k = 0; k < nblk; ++k) {
        cb.push_back({(long long)(all[k].B - bbase), (long long)k * NN, (int)all[k].ldB, N, all[k].n,
                      all[k].n});
        cv.push_back({(long long)(all[k].V - vbase), (long long)k * n * N, n, n, n, all[k].n});
      }
      copy_blocks(bbase, Bp, cb, ar, s);
      copy_blocks(vbase, Vp, cv, ar, s);
    }
    std::vector<int> nbh(nblk);
    for (int k = 0; k < nblk; ++k) nbh[k] = all[k].n;
    int* d_nb = upload(ar, nbh, s);

    // diagonal of each block (shift choice and the scalar test)
    double* d_diag = ar.dalloc((size_t)nblk * N);
    hipLaunchKernelGGL(diag_kernel, grid2(N, nblk), dim3(256), 0, s, N, Bp, d_nb, d_diag);
    ZCSD_CHECK_LAUNCH();
    std::vector<double> diag((size_t)nblk * N);
    d2h(diag.data(), d_diag, diag.size() * sizeof(double), s);
    std::vector<double> mean(nblk);
    for (int k = 0; k < nblk; ++k) {
      double t = 0.0;
      for (int i = 0; i < all[k].n; ++i) t += diag[(size_t)k * N + i];
      mean[k] = t / all[k].n;
    }
    double* d_mean = upload(ar, mean, s);
    double* d_spread = ar.dalloc(nblk);
    {
      SumsqRegion rg;
      rg.nb = d_nb;
      rg.shift = d_mean;
      rg.max_cols = N;
      sumsq_region(nblk, Bp, N, NN, rg, d_spread, ar, s);
    }
    std::vector<double> spread(nblk);
    d2h(spread.data(), d_spread, nblk * sizeof(double), s);

    // finished blocks: scalar (any basis) or leaves (Jacobi)
    std::vector<int> leaf_idx, scalar_idx, split_idx;
    for (int k = 0; k < nblk; ++k) {
      if (all[k].drop || std::sqrt(spread[k]) <= scalar_tol) scalar_idx.push_back(k);
      else if (all[k].n <= nleaf) leaf_idx.push_back(k);
      else split_idx.push_back(k);
    }
    {
      std::vector<long long> add(nprob, 0);
      for (int k : scalar_idx) add[all[k].prob] += all[k].n;
      for (int k : leaf_idx) add[all[k].prob] += all[k].n;
      for (int p = 0; p < nprob; ++p)
        if (col_out[p] + parked_cols[p] + add[p] > n)
          throw NumError(ZCSD_ENOCONV, "zolo_eig: block sizes exceed n");
    }
    // scalar blocks: V columns as they are, eigenvalues = diag
    if (!scalar_idx.empty()) {
      std::vector<CopyDesc> cv;
      for (int k : scalar_idx) {
        const int p = all[k].prob;
        cv.push_back({(long long)k * n * N, p * nn + (long long)col_out[p] * n, n, n, n, all[k].n});
        for (int i = 0; i < all[k].n; ++i) lam_out[p].push_back(diag[(size_t)k * N + i]);
        col_out[p] += all[k].n;
      }
      copy_blocks(Vp, Vout, cv, ar, s);
    }
    // leaves: parked (their blocks and bases stay in this level's buffers) and
    // solved together after the last level, one Jacobi launch for all of them
    for (int k : leaf_idx) {
      parked.push_back({Bp + (long long)k * NN, N, Vp + (long long)k * n * N, all[k].n, all[k].prob});
      parked_cols[all[k].prob] += all[k].n;
    }
    if (split_idx.empty()) {
      active.clear();
      break;
    }

    // --- split step on the remaining blocks ---------------------------------
    const int ns = (int)split_idx.size();
    // shifts and scalings (padded to the level's N; the split set is a prefix of `all`)
    std::vector<double> sh(nblk, 0.0), inva(nblk, 1.0);
    for (int q = 0; q < ns; ++q) {
      const int k = split_idx[q];
      Blk& b = all[k];
      if (!b.has_split_at) {
        // every eigenvalue of the block lies within ||B_blk - mean I||_2 <=
        // ||B_blk - mean I||_F of its mean: tighten the tracked interval.  A
        // stale end (the initial margin below a tight cluster, say) would push
        // the median out of the accepted range and leave the cluster to
        // bisection, one sign function per halving of the interval
        const double dev = std::sqrt(spread[k]) * (1.0 + 1e-10) + scalar_tol;
        const double lo2 = std::max(b.lo, mean[k] - dev), hi2 = std::min(b.hi, mean[k] + dev);
        if (lo2 < hi2) {
          b.lo = lo2;
          b.hi = hi2;
        }
      }
      std::vector<double> d(diag.begin() + (size_t)k * N, diag.begin() + (size_t)k * N + b.n);
      std::nth_element(d.begin(), d.begin() + b.n / 2, d.end());
      double sft = d[b.n / 2];
      const double w = b.hi - b.lo;
      if (b.tries > 0 || !(sft > b.lo + 1e-3 * w && sft < b.hi - 1e-3 * w)) sft = 0.5 * (b.lo + b.hi);
      if (b.has_split_at && b.tries == 0 && b.split_at > b.lo && b.split_at < b.hi) sft = b.split_at;
      sh[k] = sft;
      const double alpha = std::max(b.hi - sft, sft - b.lo) * (1.0 + 1e-12) + 1e-300;
      inva[k] = 1.0 / alpha;
    }
    // the split blocks occupy indices split_idx; gather them into a compact batch
    std::vector<int> map(ns);
    for (int q = 0; q < ns; ++q) map[q] = split_idx[q];
    int Ns = 1;
    for (int q = 0; q < ns; ++q) Ns = std::max(Ns, all[map[q]].n);
    const long long SS = (long long)Ns * Ns;
    double* Bs = ar.dalloc((size_t)ns * SS);
    double* Vs = ar.dalloc((size_t)ns * n * Ns);
    set_identity(ns, Ns, Ns, 0.0, Bs, Ns, SS, s);
    set_identity(ns, n, Ns, 0.0, Vs, n, (long long)n * Ns, s);
    {
      std::vector<CopyDesc> cb, cv;
      for (int q = 0; q < ns; ++q) {
        const int k = map[q];
        cb.push_back({(long long)k * NN, (long long)q * SS, N, Ns, all[k].n, all[k].n});
        cv.push_back({(long long)k * n * N, (long long)q * n * Ns, n, n, n, all[k].n});
      }
      copy_blocks(Bp, Bs, cb, ar, s);
      copy_blocks(Vp, Vs, cv, ar, s);
    }
    std::vector<int> nbs(ns);
    std::vector<double> shs(ns), invas(ns);
    for (int q = 0; q < ns; ++q) {
      nbs[q] = all[map[q]].n;
      shs[q] = sh[map[q]];
      invas[q] = inva[map[q]];
    }
    int* d_nbs = upload(ar, nbs, s);
    double* d_sh = upload(ar, shs, s);
    double* d_inva = upload(ar, invas, s);
    double* X = ar.dalloc((size_t)ns * SS);
    hipLaunchKernelGGL(form_shifted_kernel, grid2(SS, ns), dim3(256), 0, s, Ns, Bs, X, d_nbs, d_sh,
                       d_inva);
    ZCSD_CHECK_LAUNCH();
    double* W = ar.dalloc((size_t)ns * SS);
    {
      ZoloPdArgs za;
      za.batch = ns;
      za.n = Ns;
      za.alpha = 1.0;
      za.X = X; za.ldx = Ns; za.sx = SS;
      za.W = W; za.H = nullptr; za.X1 = nullptr;
      za.eps = a.eps; za.tol = a.tol;
      za.symmetric_input = true;
      // in the mixed mode the sign function's products run on the FP32 matrix
      // cores too (the compact-WY factors of its QRs excepted); the split only
      // needs the invariant subspaces, which the subspace-iteration step below
      // refines
      GemmFp64Scope fp64(!a.lowp);
      double t0 = 0.0;
      if (lt) {
        HostSync::sync(s);
        t0 = wall_ms();
      }
      ZoloPdResult zr = zolo_pd_batched(za, ar, s);
      res.max_r = std::max(res.max_r, zr.r);
      if (lt) {
        HostSync::sync(s);
        lt_sign = wall_ms() - t0;
        lt_r = zr.r;
        lt_ns = ns;
        lt_N = Ns;
      }
    }
    std::vector<double> offW(ns, 0.0), offY(ns, 0.0), offQ(ns, 0.0), offX(ns, 0.0);
    auto offpad = [&](const double* M, std::vector<double>& o) {
      if (!log_enabled()) return;
      double* d_o = ar.dalloc(ns);
      hipLaunchKernelGGL(offpad_kernel, dim3(ns), dim3(256), 0, s, Ns, M, d_nbs, d_o);
      ZCSD_CHECK_LAUNCH();
      d2h(o.data(), d_o, ns * sizeof(double), s);
    };
    offpad(W, offW);
    hipLaunchKernelGGL(projector_kernel, grid2(SS, ns), dim3(256), 0, s, Ns, W, d_nbs);
    ZCSD_CHECK_LAUNCH();
    double* d_tr = ar.dalloc(ns);
    hipLaunchKernelGGL(trace_real_kernel, dim3(ns), dim3(256), 0, s, Ns, W, d_nbs, d_tr);
    ZCSD_CHECK_LAUNCH();
    std::vector<double> tr(ns);
    d2h(tr.data(), d_tr, ns * sizeof(double), s);
    std::vector<int> npos(ns);
    for (int q = 0; q < ns; ++q) {
      long long v = std::llround(tr[q]);
      npos[q] = (int)std::min<long long>(std::max<long long>(v, 0), nbs[q]);
    }
    // basis: the orthogonal factor of the Householder QR of P Omega_1, Omega_1 =
    // the first kq columns of Omega, kq = the largest n+ of the level: its first
    // n+ columns span range(P) and the rest its complement, so the reflectors of
    // kq columns (not Ns) give the whole Ns x Ns factor
    int kq = 1;
    for (int q = 0; q < ns; ++q) kq = std::max(kq, npos[q]);
    double* Om = ar.dalloc((size_t)ns * SS);
    hipLaunchKernelGGL(omega_kernel, grid2(SS, ns), dim3(256), 0, s, Ns, Om, d_nbs, seed);
    ZCSD_CHECK_LAUNCH();
    seed = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    double* Y = X;  // X is dead
    {
      GemmBatch g;
      g.batch = ns;
      g.m = Ns; g.n = kq; g.k = Ns;
      g.A = W; g.lda = Ns; g.sA = SS;
      g.B = Om; g.ldb = Ns; g.sB = SS;
      g.C = Y; g.ldc = Ns; g.sC = SS;
      dgemm(g, s);
    }
    offpad(Y, offY);
    double* Q = Om;  // Omega is dead after the product
    {
      ArenaScope qs(ar);
      QRWork wk = qr_work_alloc(ar, QRShape::General, ns, Ns, kq, 32, Ns);
      geqrf_batched(ns, QRShape::General, Ns, kq, Y, Ns, SS, wk, s);
      orgqr_batched(ns, QRShape::General, Ns, kq, Q, Ns, SS, nullptr, wk, s, Ns);
    }
    offpad(Q, offQ);
    if (log_enabled())
      for (int q = 0; q < ns; ++q)
        std::fprintf(stderr, "[zcsd] eig level %d block %d n=%d N=%d off-pad |W|=%.2e |Y|=%.2e |Q|=%.2e\n",
                     res.levels, q, nbs[q], Ns, offW[q], offY[q], offQ[q]);
    // One step of subspace iteration on P.  The QR of P Omega leaves Q1 (first n+
    // columns of Q) off the eigenspace by about u kappa(V+^T Omega1), which grows
    // with n and would pass straight into the off-diagonal block of Q^T B Q.  With
    // Z = Q^T P Q, X = Z(n+:, :n+) is that coupling, and span(P Q1) is spanned by the
    // first n+ columns of Q [I -X^T; X I] (exact up to O(||X||^2) in the basis and
    // in its orthogonality); when ||X||_F is not below 2^-27 the step is taken in
    // full instead, Q <- Q factor of the QR of P Q.
    int* d_np = upload(ar, npos, s);
    double* T1 = W;  // W (P) is dead unless the subspace step below uses it
    // One block (the first level): only the coupling X = Q2^T P Q1 and the
    // diagonal blocks of Q^T B Q are needed, and the correction splits into
    // Q1 + Q2 X and Q2 - Q1 X^T (about 2.4 n^3 of the 12 n^3 dense flops saved)
    const bool one = (ns == 1 && npos[0] > 0 && npos[0] < Ns && nbs[0] == Ns);
    bool one_proj = false;
    if (one) {
      const int np = npos[0], nm = Ns - np;
      double* Q1 = Q;
      double* Q2 = Q + (long long)np * Ns;
      double* PQ = ar.dalloc((size_t)SS);
      auto mm = [&](int ta, int tb, int m_, int n_, int k_, const double* A_, const double* B_,
                    double* C_, double alpha, double beta) {
        GemmBatch g;
        g.transA = ta; g.transB = tb;
        g.m = m_; g.n = n_; g.k = k_;
        g.A = A_; g.lda = Ns; g.B = B_; g.ldb = Ns; g.C = C_; g.ldc = Ns;
        g.alpha = alpha; g.beta = beta;
        dgemm(g, s);
      };
      mm(0, 0, Ns, np, Ns, W, Q1, PQ, 1.0, 0.0);             // P Q1
      mm(1, 0, nm, np, Ns, Q2, PQ, Y + np, 1.0, 0.0);        // X = Q2^T P Q1 at Z(np:, :np)
      double xmax = 0.0;
      {
        double* d_x = ar.dalloc(1);
        SumsqRegion rg;
        rg.nb = d_nbs;
        rg.np = d_np;
        rg.max_cols = Ns;
        sumsq_region(1, Y, Ns, SS, rg, d_x, ar, s);
        double xs = 0.0;
        d2h(&xs, d_x, sizeof(double), s);
        xmax = std::sqrt(xs);
      }
      res.max_coupling = std::max(res.max_coupling, xmax);
      if (xmax <= 0x1p-27) {
        double* Qn = W;  // P is dead
        copy_scale(1, Ns, Ns, 1.0, Q, Ns, SS, Qn, Ns, SS, s);
        mm(0, 0, Ns, np, nm, Q2, Y + np, Qn, 1.0, 1.0);                         // Q1 + Q2 X
        mm(0, 1, Ns, nm, np, Q1, Y + np, Qn + (long long)np * Ns, -1.0, 1.0);  // Q2 - Q1 X^T
        Q = Qn;
        T1 = PQ;
      } else {
        ++res.full_refinements;
        mm(0, 0, Ns, nm, Ns, W, Q2, PQ + (long long)np * Ns, 1.0, 0.0);  // the rest of P Q
        ArenaScope qs(ar);
        QRWork wk = qr_work_alloc(ar, QRShape::General, 1, Ns, Ns, 32);
        geqrf_batched(1, QRShape::General, Ns, Ns, PQ, Ns, SS, wk, s);
        orgqr_batched(1, QRShape::General, Ns, Ns, Q, Ns, SS, nullptr, wk, s);
        T1 = W;
      }
      one_proj = true;
    } else {
      double* PQ = ar.dalloc((size_t)ns * SS);
      {
        GemmBatch g;
        g.batch = ns;
        g.m = Ns; g.n = Ns; g.k = Ns;
        g.A = W; g.lda = Ns; g.sA = SS;
        g.B = Q; g.ldb = Ns; g.sB = SS;
        g.C = PQ; g.ldc = Ns; g.sC = SS;
        dgemm(g, s);
        GemmBatch h = g;
        h.transA = 1;
        h.A = Q; h.B = PQ; h.C = Y;  // Z = Q^T (P Q) into the dead QR input
        dgemm(h, s);
      }
      double xmax = 0.0;
      {
        double* d_x = ar.dalloc(ns);
        SumsqRegion rg;
        rg.nb = d_nbs;
        rg.np = d_np;
        rg.max_cols = Ns;
        sumsq_region(ns, Y, Ns, SS, rg, d_x, ar, s);
        std::vector<double> xs(ns);
        d2h(xs.data(), d_x, ns * sizeof(double), s);
        for (double v : xs) xmax = std::max(xmax, std::sqrt(v));
      }
      res.max_coupling = std::max(res.max_coupling, xmax);
      if (xmax <= 0x1p-27) {
        double* K = PQ;  // P Q is dead once Z is formed
        hipLaunchKernelGGL(coupling_skew_kernel, grid2(SS, ns), dim3(256), 0, s, Ns, Y, K, d_nbs, d_np);
        ZCSD_CHECK_LAUNCH();
        double* Qn = W;  // P is dead too
        copy_scale(ns, Ns, Ns, 1.0, Q, Ns, SS, Qn, Ns, SS, s);
        GemmBatch g;
        g.batch = ns;
        g.m = Ns; g.n = Ns; g.k = Ns;
        g.A = Q; g.lda = Ns; g.sA = SS;
        g.B = K; g.ldb = Ns; g.sB = SS;
        g.C = Qn; g.ldc = Ns; g.sC = SS;
        g.beta = 1.0;
        dgemm(g, s);
        Q = Qn;
        T1 = K;
      } else {
        ++res.full_refinements;
        ArenaScope qs(ar);
        QRWork wk = qr_work_alloc(ar, QRShape::General, ns, Ns, Ns, 32);
        geqrf_batched(ns, QRShape::General, Ns, Ns, PQ, Ns, SS, wk, s);
        orgqr_batched(ns, QRShape::General, Ns, Ns, Q, Ns, SS, nullptr, wk, s);
        T1 = W;
      }
    }

    // B' = Q^T B Q, V' = V Q
    double* Bq = Y;  // Z is dead
    if (one_proj) {
      // T1 = B Q; the diagonal blocks Q1^T B Q1 and Q2^T B Q2 (upper tiles,
      // mirrored) and, when measured, the coupling block Q2^T B Q1
      const int np = npos[0], nm = Ns - np;
      GemmBatch g;
      g.m = Ns; g.n = Ns; g.k = Ns;
      g.A = Bs; g.lda = Ns;
      g.B = Q; g.ldb = Ns;
      g.C = T1; g.ldc = Ns;
      dgemm(g, s);
      auto blk = [&](int r0, int c0, int mr, int nc, bool sym) {
        GemmBatch h;
        h.transA = 1;
        h.m = mr; h.n = nc; h.k = Ns;
        h.A = Q + (long long)r0 * Ns; h.lda = Ns;
        h.B = T1 + (long long)c0 * Ns; h.ldb = Ns;
        h.C = Bq + r0 + (long long)c0 * Ns; h.ldc = Ns;
        h.sym_upper = sym;
        dgemm(h, s);
        if (sym) mirror_upper(1, mr, h.C, Ns, SS, s);
      };
      blk(0, 0, np, np, true);
      blk(np, np, nm, nm, true);
      if (a.measure_offblock || log_enabled()) blk(np, 0, nm, np, false);
      if (log_enabled()) blk(0, np, np, nm, false);  // the diagnostics compare all of Bq
    } else {
      GemmBatch g;
      g.batch = ns;
      g.m = Ns; g.n = Ns; g.k = Ns;
      g.A = Bs; g.lda = Ns; g.sA = SS;
      g.B = Q; g.ldb = Ns; g.sB = SS;
      g.C = T1; g.ldc = Ns; g.sC = SS;
      dgemm(g, s);
      GemmBatch h = g;
      h.transA = 1;
      h.A = Q; h.B = T1; h.C = Bq;
      dgemm(h, s);
      symmetrize(ns, Ns, Bq, Ns, SS, s);
    }

    double* Vq = ar.dalloc((size_t)ns * n * Ns);
    if (res.levels == 1 && Ns == n) {
      // the first level splits whole problems, whose V is the identity: V Q = Q
      copy_scale(ns, n, n, 1.0, Q, Ns, SS, Vq, n, (long long)n * Ns, s);
    } else {
      GemmBatch g;
      g.batch = ns;
      g.m = n; g.n = Ns; g.k = Ns;
      g.A = Vs; g.lda = n; g.sA = (long long)n * Ns;
      g.B = Q; g.ldb = Ns; g.sB = SS;
      g.C = Vq; g.ldc = n; g.sC = (long long)n * Ns;
      dgemm(g, s);
    }
    if (log_enabled() && nprob == 1) {
      // diagnostics: ||Q^T Q - I||_F per block of this level
      ArenaScope ds(ar);
      double* G = ar.dalloc((size_t)ns * SS);
      GemmBatch g;
      g.batch = ns;
      g.transA = 1;
      g.m = Ns; g.n = Ns; g.k = Ns;
      g.A = Q; g.lda = Ns; g.sA = SS;
      g.B = Q; g.ldb = Ns; g.sB = SS;
      g.C = G; g.ldc = Ns; g.sC = SS;
      dgemm(g, s);
      add_diag(ns, Ns, -1.0, G, Ns, SS, s);
      double* d_o = ar.dalloc(ns);
      sumsq(ns, Ns, Ns, G, Ns, SS, d_o, ar, s);
      std::vector<double> o(ns);
      d2h(o.data(), d_o, ns * sizeof(double), s);
      // invariant: Vq_b^T B Vq_b == Bq_b (B the original matrix)
      double* BV = ar.dalloc((size_t)ns * n * Ns);
      double* E = ar.dalloc((size_t)ns * SS);
      GemmBatch g1;
      g1.batch = ns;
      g1.m = n; g1.n = Ns; g1.k = n;
      g1.A = a.B; g1.lda = a.ldb; g1.sA = 0;
      g1.B = Vq; g1.ldb = n; g1.sB = (long long)n * Ns;
      g1.C = BV; g1.ldc = n; g1.sC = (long long)n * Ns;
      dgemm(g1, s);
      GemmBatch g2;
      g2.batch = ns;
      g2.transA = 1;
      g2.m = Ns; g2.n = Ns; g2.k = n;
      g2.A = Vq; g2.lda = n; g2.sA = (long long)n * Ns;
      g2.B = BV; g2.ldb = n; g2.sB = (long long)n * Ns;
      g2.C = E; g2.ldc = Ns; g2.sC = SS;
      dgemm(g2, s);
      double* d_e = ar.dalloc(ns);
      std::vector<double> ev(ns);
      // E -= Bq (only the real n_b x n_b part is meaningful)
      hipLaunchKernelGGL(sub_real_kernel, grid2(SS, ns), dim3(256), 0, s, Ns, E, Bq, d_nbs);
      ZCSD_CHECK_LAUNCH();
      sumsq(ns, Ns, Ns, E, Ns, SS, d_e, ar, s);
      d2h(ev.data(), d_e, ns * sizeof(double), s);
      // orthonormality of the incoming basis Vs and of the outgoing Vq (real columns), and of Q's real block
      auto orth_real = [&](const double* X, long long ldx, long long sx, int rows) {
        double* G = ar.dalloc((size_t)ns * SS);
        GemmBatch g;
        g.batch = ns;
        g.transA = 1;
        g.m = Ns; g.n = Ns; g.k = rows;
        g.A = X; g.lda = ldx; g.sA = sx;
        g.B = X; g.ldb = ldx; g.sB = sx;
        g.C = G; g.ldc = Ns; g.sC = SS;
        dgemm(g, s);
        std::vector<double> gh((size_t)ns * SS);
        d2h(gh.data(), G, gh.size() * sizeof(double), s);
        std::vector<double> r(ns, 0.0);
        for (int q = 0; q < ns; ++q) {
          const int m = nbs[q];
          for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) {
              const double v = gh[(size_t)q * SS + i + (size_t)j * Ns] - (i == j ? 1.0 : 0.0);
              r[q] += v * v;
            }
          r[q] = std::sqrt(r[q]);
        }
        return r;
      };
      std::vector<double> oVs = orth_real(Vs, n, (long long)n * Ns, n);
      std::vector<double> oVq = orth_real(Vq, n, (long long)n * Ns, n);
      std::vector<double> oQr = orth_real(Q, Ns, SS, Ns);
      for (int q = 0; q < ns; ++q)
        std::fprintf(stderr, "[zcsd] eig level %d block %d n=%d N=%d shift=%.6g n+=%d trace=%.6f ||QtQ-I||=%.2e ||VtBV-Bq||=%.2e orth Vs=%.2e Vq=%.2e Qreal(all rows)=%.2e\n",
                     res.levels, q, nbs[q], Ns, shs[q], npos[q], tr[q], std::sqrt(o[q]), std::sqrt(ev[q]), oVs[q], oVq[q], oQr[q]);
    }
    if (a.measure_offblock) {
      double* d_off = ar.dalloc(ns);
      SumsqRegion rg;
      rg.nb = d_nbs;
      rg.np = d_np;
      rg.max_cols = Ns;
      sumsq_region(ns, Bq, Ns, SS, rg, d_off, ar, s);
      std::vector<double> off(ns);
      d2h(off.data(), d_off, ns * sizeof(double), s);
      for (int q = 0; q < ns; ++q)
        res.max_offblock = std::max(res.max_offblock, std::sqrt(off[q]) / std::max(bnorm, 1e-300));
    }
    // children (Bq and Vq stay alive until the next level copies them)
    std::vector<Blk> next;
    for (int q = 0; q < ns; ++q) {
      const Blk& b = all[map[q]];
      const int np = npos[q];
      const double sft = shs[q];
      if (b.has_split_at && np == b.n) {
        // every eigenvalue lies above keep_below: none of them is wanted
        Blk c = b;
        c.B = Bs + q * SS;
        c.ldB = Ns;
        c.V = Vs + (long long)q * n * Ns;
        c.has_split_at = false;
        c.drop = true;
        next.push_back(c);
        continue;
      }
      if (np == 0 || np == b.n) {
        ++res.failed_splits;
        Blk c = b;
        c.has_split_at = false;
        c.B = Bs + q * SS;
        c.ldB = Ns;
        c.V = Vs + (long long)q * n * Ns;
        if (np == 0) c.hi = sft; else c.lo = sft;
        c.tries = b.tries + 1;
        if (c.tries > 60) throw NumError(ZCSD_ENOCONV, "zolo_eig: divide and conquer stalled");
        next.push_back(c);
        continue;
      }
      ++res.splits;
      Blk plus;
      plus.prob = b.prob;
      plus.n = np;
      plus.lo = sft;
      plus.hi = b.hi;
      plus.drop = b.has_split_at;  // above keep_below: not wanted
      plus.B = Bq + q * SS;
      plus.ldB = Ns;
      plus.V = Vq + (long long)q * n * Ns;
      Blk minus;
      minus.prob = b.prob;
      minus.n = b.n - np;
      minus.lo = b.lo;
      minus.hi = sft;
      minus.B = Bq + q * SS + np + (long long)np * Ns;
      minus.ldB = Ns;
      minus.V = Vq + (long long)q * n * Ns + (long long)np * n;
      next.push_back(minus);
      next.push_back(plus);
    }
    if (lt) {
      HostSync::sync(s);
      std::fprintf(stderr, "[zcsd] eig level %d: %d blocks, %d split at padded size %d, r = %d, "
                   "sign function %.2f ms, level %.2f ms\n", res.levels, lt_blocks, lt_ns, lt_N,
                   lt_r, lt_sign, wall_ms() - lt_start);
    }
    active.swap(next);
  }
  solve_leaves();
  for (int p = 0; p < nprob; ++p)
    if (col_out[p] != n) throw NumError(ZCSD_ENOCONV, "zolo_eig: lost eigenpairs");

  // sort ascending and write V, lambda (per problem)
  std::vector<CopyDesc> cv;
  cv.reserve((size_t)nprob * n);
  std::vector<double> lam_sorted((size_t)nprob * n);
  std::vector<int> perm(n);
  for (int p = 0; p < nprob; ++p) {
    const std::vector<double>& lo = lam_out[p];
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return lo[x] < lo[y]; });
    for (int j = 0; j < n; ++j) {
      cv.push_back({p * nn + (long long)perm[j] * n, p * a.sV + (long long)j * a.ldv, n, (int)a.ldv,
                    n, 1});
      lam_sorted[(size_t)p * n + j] = lo[perm[j]];
    }
  }
  copy_blocks(Vout, a.V, cv, ar, s);
  if (nprob == 1 || a.sL == n) {
    h2d(a.lam, lam_sorted.data(), (size_t)nprob * n * sizeof(double), s);
  } else {
    for (int p = 0; p < nprob; ++p)
      h2d(a.lam + p * a.sL, lam_sorted.data() + (size_t)p * n, n * sizeof(double), s);
  }
  return res;
}

}  // namespace zcsd
