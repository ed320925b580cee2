// Zolo-csd driver: Algorithm 1 (full rank) and Algorithm 3 (rank-deficient
// partial isometry) on the device, with Remarks (iii), (vi) and (vii).
//
//   rank: r_A = round(||A||_F^2) (Remark (vi)); mu = 0 if r_A = n else 2
//   polars: W_i H_i = A_i for i = 1, 2 in one batched Zolo-pd (the two polars
//       run side by side, Remark (ii)); rank-deficient inputs use the modified
//       Zolo-pd on [eps, 1] with r = 8 (Sec. 5.1, Algorithm 3)
//   B = H2 - H1 + mu (I - A1^T A1 - A2^T A2), symmetrised
//   V1 Lambda V1^T = B by Zolo-eig
//   rank-deficient: keep the eigenvectors with Lambda in [-1, 1] (Algorithm 3)
//   U_i = W_i V1
//   C = diag(V1^T H1 V1), S = diag(V1^T H2 V1)
//   theta = atan2(S_ii, C_ii) clamped to [0, pi/2] (Remark (iii)), columns
//       sorted by ascending theta.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <vector>

#include "zcsd_api_guard.h"
#include "zcsd_eig.h"
#include "zcsd_internal.h"
#include "zcsd_la.h"
#include "zcsd_zolo.h"

namespace zcsd {


// out[j] = sum_i V(i, j) T(i, j), one workgroup per column
__global__ void coldot_kernel(int n, const double* __restrict__ V, long long ldv,
                              const double* __restrict__ T, long long ldt, double* out) {
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    acc += V[i + (long long)j * ldv] * T[i + (long long)j * ldt];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

// theta_j = clamp(atan2(s_j, c_j), 0, pi/2)   (Remark (iii))
__global__ void theta_kernel(int r, const double* __restrict__ c, const double* __restrict__ s,
                             double* th) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < r) {
    double t = atan2(s[j], c[j]);
    t = fmin(fmax(t, 0.0), 1.5707963267948966);
    th[j] = t;
  }
}

// Remark (iv), the cheaper alternative to C, S from V1^T H_i V1: theta_j solves
// sin(theta) - cos(theta) = Lambda_jj, i.e. theta = pi/4 + asin(Lambda_jj / sqrt(2))
__global__ void theta_from_lambda_kernel(int r, const double* __restrict__ lam, double* th) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < r) {
    const double x = fmin(fmax(lam[j], -1.0), 1.0);
    const double t = 0.7853981633974483 + asin(x * 0.7071067811865476);
    th[j] = fmin(fmax(t, 0.0), 1.5707963267948966);
  }
}


static double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

size_t csd_workspace_bytes(int n) {
  const size_t nn = (size_t)n * n;
  // polar batch (2 problems, r <= 8), Zolo-eig levels, assembly buffers
  return (2 * 64 * nn + 64 * nn + 16 * nn) * sizeof(double) + (256u << 20);
}

// d_b[j] = -1 if R_b(j, j) < 0 else 1
__global__ void rsign_kernel(int n, const double* __restrict__ R, long long sR, double* d) {
  const long long b = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
    d[b * n + j] = (R[b * sR + j + (long long)j * n] < 0.0) ? -1.0 : 1.0;
}

// Q_b(:, j) *= d_b[j] and R_b(i, :) *= d_b[i]  (diag(R) >= 0 convention)
__global__ void rsign_apply_kernel(int n, double* Q, double* R, long long sM,
                                   const double* __restrict__ d) {
  const long long b = blockIdx.y;
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    Q[b * sM + e] *= d[b * n + j];
    R[b * sM + e] *= d[b * n + i];
  }
}

// QR with diag(R) >= 0 of the `batch` n x n matrices at M (stride n*n,
// overwritten by R) into Q
static void qr_pos(int batch, int n, double* M, double* Q, Arena& ar, hipStream_t s) {
  const long long nn = (long long)n * n;
  ArenaScope sc(ar);
  QRWork wk = qr_work_alloc(ar, QRShape::General, batch, n, n, 32);
  geqrf_batched(batch, QRShape::General, n, n, M, n, nn, wk, s);
  orgqr_batched(batch, QRShape::General, n, n, Q, n, nn, nullptr, wk, s);
  double* d = ar.dalloc((size_t)batch * n);
  const unsigned g1 = (unsigned)std::max(1, std::min((n + 255) / 256, 1024));
  hipLaunchKernelGGL(rsign_kernel, dim3(g1, batch), dim3(256), 0, s, n, M, nn, d);
  ZCSD_CHECK_LAUNCH();
  const unsigned g2 = (unsigned)std::max<long long>(1, std::min<long long>((nn + 255) / 256, 1024));
  hipLaunchKernelGGL(rsign_apply_kernel, dim3(g2, batch), dim3(256), 0, s, n, Q, M, nn, d);
  ZCSD_CHECK_LAUNCH();
}

// Algorithm 2 on both polars: W_i = Q_i Q~_i^T; returns max_i ||R~_i - R_i||_F / ||R_i||_F
// W_i = Q_i Q~_i^T is written to Wr (2 problems, n x n, stride n*n); rel[i] =
// ||R~_i - R_i||_F / ||R_i||_F
static void polar_repair(int n, const double* X, double* Wr, const double* H, double rel[2],
                         Arena& ar, hipStream_t s) {
  const long long nn = (long long)n * n;
  ArenaScope sc(ar);
  double* RA = ar.dalloc(2 * (size_t)nn);
  double* RH = ar.dalloc(2 * (size_t)nn);
  double* QA = ar.dalloc(2 * (size_t)nn);
  double* QH = ar.dalloc(2 * (size_t)nn);
  copy_scale(2, n, n, 1.0, X, n, nn, RA, n, nn, s);
  copy_scale(2, n, n, 1.0, H, n, nn, RH, n, nn, s);
  qr_pos(2, n, RA, QA, ar, s);
  qr_pos(2, n, RH, QH, ar, s);
  GemmBatch g;
  g.batch = 2;
  g.transB = 1;
  g.m = n; g.n = n; g.k = n;
  g.A = QA; g.lda = n; g.sA = nn;
  g.B = QH; g.ldb = n; g.sB = nn;
  g.C = Wr; g.ldc = n; g.sC = nn;
  dgemm(g, s);
  // ||R~ - R||_F / ||R||_F per polar (RH <- RH - RA)
  double* ss = ar.dalloc(4);
  sumsq(2, n, n, RA, n, nn, ss, ar, s);
  axpby(2 * nn, -1.0, RA, 1.0, RH, s);
  sumsq(2, n, n, RH, n, nn, ss + 2, ar, s);
  double h[4];
  d2h(h, ss, sizeof(h), s);
  rel[0] = std::sqrt(h[2] / std::max(h[0], 1e-300));
  rel[1] = std::sqrt(h[3] / std::max(h[1], 1e-300));
}

// Y1 = U1 diag(sin theta), Y2 = U2 diag(cos theta) (n x n, Y ld n)
__global__ void cs_scale_kernel(int n, const double* __restrict__ U1, long long ldu1,
                                const double* __restrict__ U2, long long ldu2,
                                const double* __restrict__ theta, double* Y1, double* Y2) {
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    const double t = theta[j];
    Y1[e] = U1[i + (long long)j * ldu1] * sin(t);
    Y2[e] = U2[i + (long long)j * ldu2] * cos(t);
  }
}

struct CsdOut {
  bool repair = false;
  double repair_resid = 0.0;
  int rank = 0;
  ZoloPdResult pd;
  ZoloEigResult eig;
  long long lowp_products = 0;  // products run on the FP32 matrix cores
  double t_polar = 0, t_B = 0, t_eig = 0, t_asm = 0;
};

// X <- X - X (X^T X - I) / 2 in FP64 (n x m, ld n): one Newton-Schulz step
// towards the nearest matrix with orthonormal columns.  The correction is
// formed from E = X^T X - I and added to X, so that only it (not X itself)
// carries the product's rounding: the result is orthonormal to about the
// rounding of X^T X
static void newton_schulz(int n, int m, double* X, Arena& ar, hipStream_t s) {
  GemmFp64Scope fp64;
  ArenaScope sc(ar);
  double* G = ar.dalloc((size_t)m * m);
  double* T = ar.dalloc((size_t)n * m);
  GemmBatch g;
  g.transA = 1;
  g.m = m; g.n = m; g.k = n;
  g.A = X; g.lda = n;
  g.B = X; g.ldb = n;
  g.C = G; g.ldc = m;
  g.sym_upper = true;
  dgemm(g, s);
  mirror_upper(1, m, G, m, 0, s);
  add_diag(1, m, -1.0, G, m, 0, s);
  GemmBatch h;
  h.m = n; h.n = m; h.k = m;
  h.A = X; h.lda = n;
  h.B = G; h.ldb = m;
  h.C = T; h.ldc = n;
  dgemm(h, s);
  axpby((long long)n * m, -0.5, T, 1.0, X, s);
}

static CsdOut csd_run(int n, const double* A1, long long lda1, const double* A2, long long lda2,
                      double* U1, long long ldu1, double* U2, long long ldu2, double* V1,
                      long long ldv1, double* theta, double* W1o, double* W2o, const zcsd_opts& o,
                      Arena& ar, hipStream_t s) {
  CsdOut out;
  const long long nn = (long long)n * n;
  ArenaScope scope(ar);
  double t0 = now_ms();
  // mixed mode (not in the paper): iteration 2 of the two polar
  // decompositions and every product of Zolo-eig on the FP32 matrix cores,
  // each followed by an FP64 Newton-Schulz step on the factor it produced;
  // the QR-form iteration 1, B and the assembly stay FP64.  The Zolotarev
  // degree is chosen as in the FP64 mode: a looser target makes each split's
  // sign function less sharp and its subspace step fall back to the full
  // second QR more often (measured slower at n = 4096).
  const bool mixed = o.prec == ZCSD_MIXED_FP32;
  const double ztol = o.tol;
  const long long lowp0 = gemm_lowp_launches();

  // rank from ||A||_F^2 (Remark (vi))
  double* X = ar.dalloc(2 * (size_t)nn);
  copy_scale(1, n, n, 1.0, A1, lda1, 0, X, n, 0, s);
  copy_scale(1, n, n, 1.0, A2, lda2, 0, X + nn, n, 0, s);
  double* d_ss = ar.dalloc(2);
  sumsq(2, n, n, X, n, nn, d_ss, ar, s);
  double ss[2];
  d2h(ss, d_ss, sizeof(ss), s);
  const double f2 = ss[0] + ss[1];
  if (!std::isfinite(f2)) throw ArgError("csd: input contains NaN or Inf");
  const long long rA = std::llround(f2);
  bool deficient;
  if (o.rank_mode == ZCSD_RANK_FULL) deficient = false;
  else if (o.rank_mode == ZCSD_RANK_DEFICIENT) deficient = true;
  else {
    if (std::fabs(f2 - (double)rA) > 0.25)
      throw NumError(ZCSD_ENOTISO, "csd: ||A||_F^2 is not close to an integer rank");
    deficient = rA < n;
  }
  const double mu = deficient ? o.mu : 0.0;

  // the two polar decompositions, batched
  double* W = ar.dalloc(2 * (size_t)nn);
  double* H = ar.dalloc(2 * (size_t)nn);
  {
    ZoloPdArgs za;
    za.batch = 2;
    za.n = n;
    za.alpha = 1.0;
    za.X = X; za.ldx = n; za.sx = nn;
    za.W = W; za.H = H;
    za.eps = o.eps; za.tol = ztol;
    za.r_override = o.r_override;
    za.ell_override = o.ell_override;
    za.lowp_iter2 = mixed;
    if (deficient) {
      if (za.ell_override <= 0.0) za.ell_override = o.eps;
      if (za.r_override <= 0) za.r_override = ZOLO_RMAX;
    }
    out.pd = zolo_pd_batched(za, ar, s);
  }
  // Algorithm 2 (Sec. 5.1): a full-rank A_i whose sigma_min estimate fell to eps
  // was handled by the modified Zolo-pd, so W~_i is not orthonormal; with
  // A_i = Q_i R_i and H~_i = Q~_i R~_i (diag(R) >= 0, where the two R factors
  // agree in exact arithmetic) W_i = Q_i Q~_i^T is orthonormal by construction
  // and ||W_i H~_i - A_i|| = ||R~_i - R_i||, checked against 100 n u ||R_i||_F.
  // The rank-deficient path always runs the modified Zolo-pd, and its nonzero
  // singular values may lie below eps as well (A rank deficient and C or S
  // ill conditioned): Sec. 5.2 then takes the same lines of Algorithm 2.  There
  // the repaired W_i is kept aside and used for U_i when U_i = W~_i V_1r comes
  // out far from orthonormal (below).
  const double rep_tol = 100.0 * n * 0x1p-53;
  double* Wrep = nullptr;
  bool rep_ok[2] = {false, false};
  double rep_rel[2] = {0.0, 0.0};
  if (deficient) {
    Wrep = ar.dalloc(2 * (size_t)nn);
    polar_repair(n, X, Wrep, H, rep_rel, ar, s);
    rep_ok[0] = rep_rel[0] <= rep_tol;
    rep_ok[1] = rep_rel[1] <= rep_tol;
  } else if (out.pd.ell <= o.eps * (1.0 + 1e-12)) {
    ArenaScope rs(ar);
    double* Wr = ar.dalloc(2 * (size_t)nn);
    polar_repair(n, X, Wr, H, rep_rel, ar, s);
    out.repair = true;
    out.repair_resid = std::max(rep_rel[0], rep_rel[1]);
    if (!(out.repair_resid <= rep_tol))
      throw NumError(ZCSD_EREPAIR, "csd: ill-conditioned repair rejected (||R~ - R|| too large)");
    copy_scale(2, n, n, 1.0, Wr, n, nn, W, n, nn, s);
  }
  HostSync::sync(s);
  double t1 = now_ms();
  out.t_polar = t1 - t0;

  // B = H2 - H1 + mu (I - A^T A)
  double* B = ar.dalloc(nn);
  copy_scale(1, n, n, 1.0, H + nn, n, 0, B, n, 0, s);
  axpby(nn, -1.0, H, 1.0, B, s);
  if (mu != 0.0) {
    add_diag(1, n, mu, B, n, 0, s);
    GemmBatch g;
    g.transA = 1; g.transB = 0;
    g.m = n; g.n = n; g.k = n;
    g.A = X; g.lda = n; g.B = X; g.ldb = n;
    g.C = B; g.ldc = n;
    g.alpha = -mu; g.beta = 1.0;
    dgemm(g, s);
    g.A = X + nn; g.B = X + nn;
    dgemm(g, s);
  }
  symmetrize(1, n, B, n, 0, s);
  HostSync::sync(s);
  double t2 = now_ms();
  out.t_B = t2 - t1;

  // Zolo-eig of B
  double* V = ar.dalloc(nn);
  double* lam = ar.dalloc(n);
  {
    ZoloEigArgs ea;
    ea.n = n;
    ea.B = B; ea.ldb = n;
    const double margin = 1e-6;
    ea.lo = -1.0 - margin;
    ea.hi = (mu > 1.0 ? mu : 1.0) + margin;
    ea.V = V; ea.ldv = n;
    ea.lam = lam;
    ea.n_leaf = o.n_leaf;
    ea.eps = o.eps; ea.tol = ztol;
    ea.lowp = mixed;
    // Alg. 3 keeps only the eigenpairs in [-1, 1]: the divide and conquer
    // splits first between 1 and mu and does not divide the part at mu
    if (deficient && mu > 1.0) ea.keep_below = 0.5 * (1.0 + mu);
    out.eig = zolo_eig(ea, ar, s);
    // the basis from the FP32 products is orthonormal only to the FP32 level
    if (mixed) newton_schulz(n, n, V, ar, s);
  }
  HostSync::sync(s);
  double t3 = now_ms();
  out.t_eig = t3 - t2;

  // rank-deficient selection (eigenvalues ascending: the kept ones come first)
  int r = n;
  if (deficient) {
    std::vector<double> lh(n);
    d2h(lh.data(), lam, n * sizeof(double), s);
    r = 0;
    for (int j = 0; j < n; ++j)
      if (lh[j] <= 0.5 * (1.0 + mu)) ++r;
  }
  out.rank = r;

  // U_i = W_i V, c = diag(V^T H1 V), s = diag(V^T H2 V)
  double* Ut = ar.dalloc(2 * (size_t)nn);
  double* T = ar.dalloc(2 * (size_t)nn);
  double* cs = ar.dalloc(2 * (size_t)n);
  double* th = ar.dalloc(n);
  if (r > 0) {
    GemmBatch g;
    g.batch = 2;
    g.m = n; g.n = r; g.k = n;
    g.A = W; g.lda = n; g.sA = nn;
    g.B = V; g.ldb = n; g.sB = 0;
    g.C = Ut; g.ldc = n; g.sC = nn;
    dgemm(g, s);
    if (deficient) {
      // Newton-Schulz steps U <- U + U (I - U^T U) / 2 on U_i = W~_i V_1r.  In
      // exact arithmetic U_i is orthonormal (Sec. 5.2); in floating point the
      // zero singular values of A_i become O(u), the modified Zolo-pd maps them
      // to values strictly between 0 and 1, and when A_i also has singular
      // values only a few orders above eps the two groups mix at second order.
      // The defect U^T U - I then lives on the columns whose C_ii (or S_ii) is
      // ~0, so the correction leaves A1 = U1 C V1^T, A2 = U2 S V1^T unchanged
      // to first order.
      double* Gr = T;  // r x r per polar, T is free until the H_i V product below
      double* Tc = ar.dalloc(2 * (size_t)nn);
      if (rep_ok[0] || rep_ok[1]) {
        // ||U_i^T U_i - I||_F; beyond 1e-6 (more than the two steps below can
        // remove) U_i is taken from the repaired W_i of Algorithm 2 instead
        GemmBatch q;
        q.batch = 2;
        q.transA = 1; q.transB = 0;
        q.m = r; q.n = r; q.k = n;
        q.A = Ut; q.lda = n; q.sA = nn;
        q.B = Ut; q.ldb = n; q.sB = nn;
        q.C = Gr; q.ldc = r; q.sC = nn;
        dgemm(q, s);
        add_diag(2, r, -1.0, Gr, r, nn, s);
        double* dd = ar.dalloc(2);
        sumsq(2, r, r, Gr, r, nn, dd, ar, s);
        double hd[2];
        d2h(hd, dd, sizeof(hd), s);
        for (int i = 0; i < 2; ++i) {
          if (rep_ok[i] && hd[i] > 1e-12) {
            GemmBatch w;
            w.m = n; w.n = r; w.k = n;
            w.A = Wrep + i * nn; w.lda = n;
            w.B = V; w.ldb = n;
            w.C = Ut + i * nn; w.ldc = n;
            dgemm(w, s);
            out.repair = true;
            out.repair_resid = std::max(out.repair_resid, rep_rel[i]);
          }
        }
      }
      for (int it = 0; it < 2; ++it) {
        GemmBatch q;
        q.batch = 2;
        q.transA = 1; q.transB = 0;
        q.m = r; q.n = r; q.k = n;
        q.A = Ut; q.lda = n; q.sA = nn;
        q.B = Ut; q.ldb = n; q.sB = nn;
        q.C = Gr; q.ldc = r; q.sC = nn;
        dgemm(q, s);
        GemmBatch u;
        u.batch = 2;
        u.m = n; u.n = r; u.k = r;
        u.A = Ut; u.lda = n; u.sA = nn;
        u.B = Gr; u.ldb = r; u.sB = nn;
        u.C = Tc; u.ldc = n; u.sC = nn;
        dgemm(u, s);
        axpby((long long)n * r, -0.5, Tc, 1.5, Ut, s);
        axpby((long long)n * r, -0.5, Tc + nn, 1.5, Ut + nn, s);
      }
    }
    if (o.postprocess == 2) {
      // Remark (iv): theta from the eigenvalues (the kept ones lie in [-1, 1])
      hipLaunchKernelGGL(theta_from_lambda_kernel, dim3((r + 255) / 256), dim3(256), 0, s, r, lam,
                         th);
      ZCSD_CHECK_LAUNCH();
    } else {
      g.A = H;
      g.C = T;
      dgemm(g, s);
      hipLaunchKernelGGL(coldot_kernel, dim3(r), dim3(256), 0, s, n, V, (long long)n, T,
                         (long long)n, cs);
      ZCSD_CHECK_LAUNCH();
      hipLaunchKernelGGL(coldot_kernel, dim3(r), dim3(256), 0, s, n, V, (long long)n, T + nn,
                         (long long)n, cs + n);
      ZCSD_CHECK_LAUNCH();
      hipLaunchKernelGGL(theta_kernel, dim3((r + 255) / 256), dim3(256), 0, s, r, cs, cs + n, th);
      ZCSD_CHECK_LAUNCH();
    }
  }
  // order by ascending theta and write the outputs (columns r..n-1 zero)
  std::vector<double> thh(r);
  if (r > 0) d2h(thh.data(), th, r * sizeof(double), s);
  std::vector<int> perm(r);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return thh[x] < thh[y]; });
  set_identity(1, n, n, 0.0, U1, ldu1, 0, s);
  set_identity(1, n, n, 0.0, U2, ldu2, 0, s);
  set_identity(1, n, n, 0.0, V1, ldv1, 0, s);
  std::vector<double> th_sorted(n, 0.0);
  {
    std::vector<CopyDesc> c1, c2, c3;
    for (int j = 0; j < r; ++j) {
      c1.push_back({(long long)perm[j] * n, (long long)j * ldu1, n, (int)ldu1, n, 1});
      c2.push_back({nn + (long long)perm[j] * n, (long long)j * ldu2, n, (int)ldu2, n, 1});
      c3.push_back({(long long)perm[j] * n, (long long)j * ldv1, n, (int)ldv1, n, 1});
      th_sorted[j] = thh[perm[j]];
    }
    copy_blocks(Ut, U1, c1, ar, s);
    copy_blocks(Ut, U2, c2, ar, s);
    copy_blocks(V, V1, c3, ar, s);
  }
  h2d(theta, th_sorted.data(), n * sizeof(double), s);
  if (W1o) copy_scale(1, n, n, 1.0, W, n, 0, W1o, n, 0, s);
  if (W2o) copy_scale(1, n, n, 1.0, W + nn, n, 0, W2o, n, 0, s);
  HostSync::sync(s);
  out.t_asm = now_ms() - t3;
  out.lowp_products = gemm_lowp_launches() - lowp0;
  return out;
}

// One problem of a batch through the single path (Algorithm 2 included):
// U1, U2, V1 (n x n, ld n) and theta (n) on the device, the rank returned.
int csd_single_member(int n, const double* A1, const double* A2, double* U1, double* U2,
                      double* V1, double* theta, const zcsd_opts& o, Arena& ar, hipStream_t s,
                      bool* repaired) {
  CsdOut r = csd_run(n, A1, n, A2, n, U1, n, U2, n, V1, n, theta, nullptr, nullptr, o, ar, s);
  if (repaired) *repaired = r.repair;
  return r.rank;
}

}  // namespace zcsd

using namespace zcsd;

static void fill_csd_info(zcsd_info* info, const CsdOut& r) {
  if (!info) return;
  *info = zcsd_info{};
  info->rank = r.rank;
  info->r_used[0] = info->r_used[1] = r.pd.r;
  info->ell[0] = info->ell[1] = r.pd.ell;
  info->zolo_resid = r.pd.resid;
  info->eig_levels = r.eig.levels;
  info->eig_splits = r.eig.splits;
  info->eig_max_r = r.eig.max_r;
  info->eig_offblock = r.eig.max_offblock;
  info->eig_coupling = r.eig.max_coupling;
  info->eig_full_refinements = r.eig.full_refinements;
  info->lowp_products = (int)std::min<long long>(r.lowp_products, 1 << 30);
  info->repair = r.repair ? 1 : 0;
  info->repair_resid = r.repair_resid;
  info->time_ms[0] = r.t_polar;
  info->time_ms[1] = r.t_B;
  info->time_ms[2] = r.t_eig;
  info->time_ms[3] = r.t_asm;
}

static void check_csd_opts(const zcsd_opts& o) {
  ZCSD_REQUIRE(o.postprocess >= 0 && o.postprocess <= 2, "csd: postprocess must be 0, 1 or 2");
  ZCSD_REQUIRE(o.r_override >= 0 && o.r_override <= ZOLO_RMAX, "csd: r_override out of range");
  ZCSD_REQUIRE(o.prec == ZCSD_FP64 || o.prec == ZCSD_MIXED_FP32, "csd: unknown precision mode");
  ZCSD_REQUIRE(o.eps > 0.0 && o.eps < 1.0 && o.tol > 0.0, "csd: eps/tol out of range");
  ZCSD_REQUIRE(o.mu > 1.0 || o.rank_mode == ZCSD_RANK_FULL, "csd: mu must exceed 1");
}

extern "C" zcsd_status zcsd_dcsd(zcsd_handle* handle, int n, const double* d_A1, int lda1,
                                 const double* d_A2, int lda2, double* d_U1, int ldu1, double* d_U2,
                                 int ldu2, double* d_V1, int ldv1, double* d_theta, double* d_W1,
                                 double* d_W2, const zcsd_opts* opts, zcsd_info* info) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(n >= 1, "csd: n must be positive");
    ZCSD_REQUIRE(d_A1 && d_A2 && d_U1 && d_U2 && d_V1 && d_theta, "csd: NULL pointer");
    ZCSD_REQUIRE(lda1 >= n && lda2 >= n && ldu1 >= n && ldu2 >= n && ldv1 >= n,
                 "csd: leading dimension < n");
    zcsd_opts o;
    zcsd_default_opts(&o);
    if (opts) o = *opts;
    check_csd_opts(o);
    ZCSD_HIP(hipSetDevice(handle->device));
    handle->arena.reset();
    handle->arena.reserve(csd_workspace_bytes(n));
    CsdOut r = csd_run(n, d_A1, lda1, d_A2, lda2, d_U1, ldu1, d_U2, ldu2, d_V1, ldv1, d_theta,
                       d_W1, d_W2, o, handle->arena, handle->stream);
    fill_csd_info(info, r);
  });
}

extern "C" zcsd_status zcsd_workspace_size(zcsd_handle* handle, int n, const zcsd_opts* opts,
                                           size_t* bytes) {
  (void)handle;
  return guarded([&] {
    ZCSD_REQUIRE(n >= 1, "workspace_size: n must be positive");
    ZCSD_REQUIRE(bytes != nullptr, "workspace_size: NULL pointer");
    zcsd_opts o;
    zcsd_default_opts(&o);
    if (opts) o = *opts;
    check_csd_opts(o);
    *bytes = csd_workspace_bytes(n);
  });
}

// Householder QR of the m x n block A (m >= n): Q (m x n, ld m) and the n x n
// triangular factor R (ld n; geqrf leaves zeros below the diagonal)
void zcsd::tall_qr(int m, int n, const double* A, long long lda, double* Q, double* R, Arena& ar,
                   hipStream_t s) {
  ArenaScope sc(ar);
  const long long mn = (long long)m * n;
  double* M = ar.dalloc((size_t)mn);
  copy_scale(1, m, n, 1.0, A, lda, 0, M, m, 0, s);
  QRWork wk = qr_work_alloc(ar, QRShape::General, 1, m, n, 32);
  geqrf_batched(1, QRShape::General, m, n, M, m, mn, wk, s);
  orgqr_batched(1, QRShape::General, m, n, Q, m, mn, nullptr, wk, s);
  copy_scale(1, n, n, 1.0, M, m, 0, R, n, 0, s);
}

// Algorithm 1 / 3 for rectangular blocks A1 (m1 x n), A2 (m2 x n), m1, m2 >= n.
// With A_i = Q_i R_i, [R1; R2] is a 2n x n partial isometry of the same rank
// with the same angles and V1, and polar(A_i) = Q_i polar(R_i): the square
// path runs on [R1; R2] and U_i = Q_i U_i'.
extern "C" zcsd_status zcsd_dcsd_mn(zcsd_handle* handle, int m1, int m2, int n,
                                    const double* d_A1, int lda1, const double* d_A2, int lda2,
                                    double* d_U1, int ldu1, double* d_U2, int ldu2, double* d_V1,
                                    int ldv1, double* d_theta, const zcsd_opts* opts,
                                    zcsd_info* info) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(n >= 1 && m1 >= n && m2 >= n, "csd_mn: need n >= 1 and m1, m2 >= n");
    ZCSD_REQUIRE(d_A1 && d_A2 && d_U1 && d_U2 && d_V1 && d_theta, "csd_mn: NULL pointer");
    ZCSD_REQUIRE(lda1 >= m1 && lda2 >= m2 && ldu1 >= m1 && ldu2 >= m2 && ldv1 >= n,
                 "csd_mn: leading dimension too small");
    zcsd_opts o;
    zcsd_default_opts(&o);
    if (opts) o = *opts;
    check_csd_opts(o);
    ZCSD_HIP(hipSetDevice(handle->device));
    const int mx = std::max(m1, m2);
    const size_t nn = (size_t)n * n;
    const size_t extra = sizeof(double) * ((size_t)(m1 + m2) * n + 4 * nn + (size_t)mx * n) +
                         qr_work_bytes(QRShape::General, 1, mx, n, 32) + (64u << 20);
    Arena& ar = handle->arena;
    ar.reset();
    ar.reserve(csd_workspace_bytes(n) + extra);
    hipStream_t s = handle->stream;
    ArenaScope scope(ar);
    double* Q1 = ar.dalloc((size_t)m1 * n);
    double* Q2 = ar.dalloc((size_t)m2 * n);
    double* R = ar.dalloc(2 * nn);   // R1, R2
    double* Up = ar.dalloc(2 * nn);  // U1', U2'
    tall_qr(m1, n, d_A1, lda1, Q1, R, ar, s);
    tall_qr(m2, n, d_A2, lda2, Q2, R + nn, ar, s);
    CsdOut r = csd_run(n, R, n, R + nn, n, Up, n, Up + nn, n, d_V1, ldv1, d_theta, nullptr,
                       nullptr, o, ar, s);
    GemmBatch g;
    g.m = m1; g.n = n; g.k = n;
    g.A = Q1; g.lda = m1;
    g.B = Up; g.ldb = n;
    g.C = d_U1; g.ldc = ldu1;
    dgemm(g, s);
    g.m = m2;
    g.A = Q2; g.lda = m2;
    g.B = Up + nn;
    g.C = d_U2; g.ldc = ldu2;
    dgemm(g, s);
    ZCSD_HIP(hipStreamSynchronize(s));
    fill_csd_info(info, r);
  });
}

extern "C" zcsd_status zcsd_dcsd2x2(zcsd_handle* handle, int n, const double* d_A1, int lda1,
                                    const double* d_A2, int lda2, const double* d_A3, int lda3,
                                    const double* d_A4, int lda4, double* d_U1, int ldu1,
                                    double* d_U2, int ldu2, double* d_V1, int ldv1, double* d_V2,
                                    int ldv2, double* d_theta, const zcsd_opts* opts,
                                    zcsd_info* info) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(n >= 1, "csd2x2: n must be positive");
    ZCSD_REQUIRE(d_A1 && d_A2 && d_A3 && d_A4 && d_U1 && d_U2 && d_V1 && d_V2 && d_theta,
                 "csd2x2: NULL pointer");
    ZCSD_REQUIRE(lda1 >= n && lda2 >= n && lda3 >= n && lda4 >= n && ldu1 >= n && ldu2 >= n &&
                     ldv1 >= n && ldv2 >= n,
                 "csd2x2: leading dimension < n");
    zcsd_opts o;
    zcsd_default_opts(&o);
    if (opts) o = *opts;
    ZCSD_REQUIRE(o.r_override >= 0 && o.r_override <= ZOLO_RMAX, "csd2x2: r_override out of range");
    ZCSD_REQUIRE(o.prec == ZCSD_FP64 || o.prec == ZCSD_MIXED_FP32, "csd2x2: unknown precision mode");
    ZCSD_REQUIRE(o.eps > 0.0 && o.eps < 1.0 && o.tol > 0.0, "csd2x2: eps/tol out of range");
    ZCSD_REQUIRE(o.rank_mode != ZCSD_RANK_DEFICIENT, "csd2x2: the first block column has full rank");
    ZCSD_REQUIRE(o.postprocess >= 0 && o.postprocess <= 2, "csd2x2: postprocess must be 0, 1 or 2");
    ZCSD_HIP(hipSetDevice(handle->device));
    handle->arena.reset();
    handle->arena.reserve(csd_workspace_bytes(n));
    hipStream_t s = handle->stream;
    CsdOut r = csd_run(n, d_A1, lda1, d_A2, lda2, d_U1, ldu1, d_U2, ldu2, d_V1, ldv1, d_theta,
                       nullptr, nullptr, o, handle->arena, s);
    if (r.rank < n)
      throw NumError(ZCSD_ENOTISO, "csd2x2: [A1; A2] is rank deficient, A is not orthogonal");
    // X = -A3^T U1 S + A4^T U2 C, V2 = Q of X = QR (diag(R) >= 0)
    Arena& ar = handle->arena;
    ArenaScope scope(ar);
    const long long nn = (long long)n * n;
    double* Y = ar.dalloc(2 * (size_t)nn);
    double* X = ar.dalloc((size_t)nn);
    double* Q = ar.dalloc((size_t)nn);
    const unsigned g = (unsigned)std::max<long long>(1, std::min<long long>((nn + 255) / 256, 4096));
    hipLaunchKernelGGL(cs_scale_kernel, dim3(g), dim3(256), 0, s, n, d_U1, (long long)ldu1, d_U2,
                       (long long)ldu2, d_theta, Y, Y + nn);
    ZCSD_CHECK_LAUNCH();
    GemmBatch gm;
    gm.transA = 1;
    gm.m = n; gm.n = n; gm.k = n;
    gm.A = d_A3; gm.lda = lda3;
    gm.B = Y; gm.ldb = n;
    gm.C = X; gm.ldc = n;
    gm.alpha = -1.0; gm.beta = 0.0;
    dgemm(gm, s);
    gm.A = d_A4; gm.lda = lda4;
    gm.B = Y + nn;
    gm.alpha = 1.0; gm.beta = 1.0;
    dgemm(gm, s);
    qr_pos(1, n, X, Q, ar, s);
    copy_scale(1, n, n, 1.0, Q, n, 0, d_V2, ldv2, 0, s);
    ZCSD_HIP(hipStreamSynchronize(s));
    if (info) {
      *info = zcsd_info{};
      info->rank = r.rank;
      info->r_used[0] = info->r_used[1] = r.pd.r;
      info->ell[0] = info->ell[1] = r.pd.ell;
      info->zolo_resid = r.pd.resid;
      info->eig_levels = r.eig.levels;
      info->eig_splits = r.eig.splits;
      info->eig_max_r = r.eig.max_r;
      info->eig_offblock = r.eig.max_offblock;
      info->repair = r.repair ? 1 : 0;
      info->repair_resid = r.repair_resid;
      info->time_ms[0] = r.t_polar;
      info->time_ms[1] = r.t_B;
      info->time_ms[2] = r.t_eig;
      info->time_ms[3] = r.t_asm;
    }
  });
}

extern "C" zcsd_status zcsd_dsyev_zolo(zcsd_handle* handle, int n, const double* d_B, int ldb,
                                       double lo, double hi, double* d_V, int ldv,
                                       double* d_lambda, const zcsd_opts* opts, zcsd_info* info) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(n >= 1, "syev: n must be positive");
    ZCSD_REQUIRE(d_B && d_V && d_lambda, "syev: NULL pointer");
    ZCSD_REQUIRE(ldb >= n && ldv >= n, "syev: leading dimension < n");
    ZCSD_REQUIRE(lo < hi && std::isfinite(lo) && std::isfinite(hi), "syev: need lo < hi");
    zcsd_opts o;
    zcsd_default_opts(&o);
    if (opts) o = *opts;
    ZCSD_HIP(hipSetDevice(handle->device));
    handle->arena.reset();
    handle->arena.reserve(csd_workspace_bytes(n));
    ZoloEigArgs ea;
    ea.n = n;
    ea.B = d_B; ea.ldb = ldb;
    ea.lo = lo; ea.hi = hi;
    ea.V = d_V; ea.ldv = ldv;
    ea.lam = d_lambda;
    ea.n_leaf = o.n_leaf;
    ea.eps = o.eps; ea.tol = o.tol;
    ZoloEigResult r = zolo_eig(ea, handle->arena, handle->stream);
    ZCSD_HIP(hipStreamSynchronize(handle->stream));
    if (info) {
      *info = zcsd_info{};
      info->rank = n;
      info->eig_levels = r.levels;
      info->eig_splits = r.splits;
      info->eig_max_r = r.max_r;
      info->eig_offblock = r.max_offblock;
      info->eig_coupling = r.max_coupling;
      info->eig_full_refinements = r.full_refinements;
    }
  });
}
