// Zolo-pd (Sec. 5): the polar decomposition X = W H in two Zolotarev steps.
//
// Every iterate keeps the singular vectors of X, X_k = P r_k(Sigma) Q^T, so
// the iteration can run on the triangular factor of a QR of X:
// X/alpha = Q R  =>  polar(X/alpha) = Q polar(R).  The device path is
//
//   0. Q R = X/alpha (blocked Householder).  l <= sigma_min(R) from
//      sigma_min >= 1/||R^{-1}||_F (R^{-1} by the level-parallel trtri),
//      floored at eps (the modified Zolo-pd of Sec. 5.1); r = smallest degree
//      with 1 - l_2 <= tol.
//   1. QR form on R (every term j = 1..r in one batch):
//        [R; sqrt(c_{2j-1}) I] = [Q1; Q2] R~  (structured QR, 2n^3/3 flops),
//        R (R^T R + c I)^{-1} = Q1 Q2^T / sqrt(c),
//        Y1 = M (R + sum_j (a_j / sqrt(c_{2j-1})) Q1_j Q2_j^T)
//      where sqrt(a_j / sqrt(c_{2j-1})) scales the [I; 0] that Q formation
//      starts from, so the r products are one GEMM with inner size r n.
//   2. Cholesky form on Y1 (well conditioned after step 1):
//        G = Y1^T Y1,  R_j^T R_j = (G + c_{2j-1} I) / a_j,
//        sum_j a_j (G + c_{2j-1} I)^{-1} = sum_j R_j^{-1} R_j^{-T},
//        Y2 = M (Y1 + Y1 sum_j R_j^{-1} R_j^{-T}).
//   3. W = Q Y2,  H = alpha sym(Y2^T R) (= sym(W^T X)); Q itself is formed
//      on a second stream during steps 1 and 2.
#include <algorithm>
#include <cmath>
#include <vector>

#include "zcsd_internal.h"
#include "zcsd_la.h"
#include "zcsd_zolo.h"

namespace zcsd {

struct Coef8 {
  double v[ZOLO_RMAX];
};

// S_{b,j} = [upper(R_b); sqrtc_j I]  (2n x n, ld 2n), problem index p = b*r + j
__global__ void stack_build_kernel(int n, int r, const double* __restrict__ R, long long ldr,
                                   long long sR, double* S, Coef8 sqrtc) {
  const long long p = blockIdx.y;
  const long long b = p / r;
  const int j = (int)(p % r);
  const long long total = 2LL * n * n;
  double* Sp = S + p * total;
  const double* Rb = R + b * sR;
  const double d = sqrtc.v[j];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % (2 * n)), col = (int)(e / (2 * n));
    double v;
    if (i < n) v = (i <= col) ? Rb[i + (long long)col * ldr] : 0.0;
    else v = (i - n == col) ? d : 0.0;
    Sp[e] = v;
  }
}

// E_{b,j} = (G_b + c_j I) * inva_j   (n x n, ld n)
__global__ void shift_scale_kernel(int n, int r, const double* __restrict__ G, double* E, Coef8 c,
                                   Coef8 inva) {
  const long long p = blockIdx.y;
  const long long b = p / r;
  const int j = (int)(p % r);
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), col = (int)(e / n);
    double v = G[b * nn + e];
    if (i == col) v += c.v[j];
    E[p * nn + e] = v * inva.v[j];
  }
}

// Ms_b = sum_j T_{b,j} on the upper triangle (i <= j), terms in order j = 0..r-1
__global__ void sum_terms_upper_kernel(int n, int r, const double* __restrict__ T, double* Ms) {
  const long long b = blockIdx.y;
  const long long nn = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), col = (int)(e / n);
    if (i > col) continue;
    double acc = 0.0;
    for (int j = 0; j < r; ++j) acc += T[(b * r + j) * nn + e];
    Ms[b * nn + e] = acc;
  }
}

static dim3 grid_for(long long total, int batch) {
  long long g = (total + 255) / 256;
  g = std::max<long long>(1, std::min<long long>(g, 2048));
  return dim3((unsigned)g, (unsigned)batch);
}

ZoloPdResult zolo_pd_batched(const ZoloPdArgs& a, Arena& ar, hipStream_t s) {
  const int B = a.batch, n = a.n;
  ZCSD_REQUIRE(B >= 1 && n >= 1, "zolo_pd: empty problem");
  const long long nn = (long long)n * n;
  ArenaScope scope(ar);
  ZoloPdResult res;

  // 0. Q R = X / alpha
  double* M = ar.dalloc((size_t)B * nn);
  copy_scale(B, n, n, 1.0 / a.alpha, a.X, a.ldx, a.sx, M, n, nn, s);
  const int nb = a.nb_qr;
  QRWork wk0 = qr_work_alloc(ar, QRShape::General, B, n, n, nb);
  geqrf_batched(B, QRShape::General, n, n, M, n, nn, wk0, s);
  // Q is needed only in step 3: it is formed on a second stream while the
  // latency-bound QRs and Cholesky factorizations of steps 1 and 2 run on s
  // (only wk0, Q and the reflectors are touched there; both live to the end)
  double* Q = ar.dalloc((size_t)B * nn);
  AuxStream side(s);
  orgqr_batched(B, QRShape::General, n, n, Q, n, nn, nullptr, wk0, side.get());

  // lower bound l
  double ell;
  if (a.ell_override > 0.0) {
    ell = a.ell_override;
  } else {
    double* Ri = ar.dalloc((size_t)B * nn);
    trtri_upper_batched(B, n, M, n, nn, Ri, n, nn, ar, s);
    double* d_ss = ar.dalloc(B);
    sumsq(B, n, n, Ri, n, nn, d_ss, ar, s);
    std::vector<double> ss(B);
    d2h(ss.data(), d_ss, B * sizeof(double), s);
    ell = 1.0;
    for (int b = 0; b < B; ++b) {
      const double v = ss[b];
      double lb = (std::isfinite(v) && v > 0.0) ? 1.0 / std::sqrt(v) : 0.0;
      ell = std::min(ell, lb);
    }
    ell *= 0.9;  // margin for the rounding of R^{-1}
  }
  ell = std::min(1.0, std::max(ell, a.eps));
  int r = a.r_override;
  if (r <= 0) {
    r = zolo_choose_r(ell, a.tol);
    if (r == 0) r = ZOLO_RMAX;
  }
  const ZoloPlan plan = zolo_plan(ell, r);
  res.r = r;
  res.ell = ell;
  res.resid = plan.resid;
  res.n_qr_terms = r;

  // 1. QR form on R
  const ZoloStepCoef& z1 = plan.step[0];
  Coef8 sqrtc{};
  std::vector<double> qscale((size_t)B * r);
  for (int j = 0; j < r; ++j) {
    sqrtc.v[j] = std::sqrt(z1.c[2 * j]);
    const double sc = std::sqrt(z1.a[j] / sqrtc.v[j]);
    for (int b = 0; b < B; ++b) qscale[(size_t)b * r + j] = sc;
  }
  const int P = B * r;
  const long long s2 = 2LL * nn;
  double* S = ar.dalloc((size_t)P * s2);
  hipLaunchKernelGGL(stack_build_kernel, grid_for(s2, P), dim3(256), 0, s, n, r, M, (long long)n,
                     nn, S, sqrtc);
  ZCSD_CHECK_LAUNCH();
  {
    ArenaScope sc1(ar);
    QRWork wk1 = qr_work_alloc(ar, QRShape::Stacked, P, 2 * n, n, nb);
    geqrf_batched(P, QRShape::Stacked, 2 * n, n, S, 2 * n, s2, wk1, s);
    double* d_qs = ar.dalloc(P);
    h2d(d_qs, qscale.data(), P * sizeof(double), s);
    orgqr_batched(P, QRShape::Stacked, 2 * n, n, S, 2 * n, s2, d_qs, wk1, s);
  }
  double* Y1 = ar.dalloc((size_t)B * nn);
  copy_scale(B, n, n, 1.0, M, n, nn, Y1, n, nn, s);
  {
    GemmBatch g;
    g.batch = B;
    g.transA = 0; g.transB = 1;
    g.m = n; g.n = n; g.k = r * n;
    g.A = S; g.lda = 2 * n; g.sA = (long long)r * s2;
    g.B = S + n; g.ldb = 2 * n; g.sB = (long long)r * s2;
    g.C = Y1; g.ldc = n; g.sC = nn;
    g.alpha = z1.M; g.beta = z1.M;
    // both factors of each term are upper triangular (Q2 = sqrt(c) R~^{-1},
    // Q1 = R R~^{-1}): only k >= max(i, j) contributes
    g.tri = 1 | 8; g.kseg = n;
    dgemm(g, s);
  }

  // 2. Cholesky form on Y1 (well conditioned: its products may run in FP32)
  const ZoloStepCoef& z2 = plan.step[1];
  double* Y2 = ar.dalloc((size_t)B * nn);
  {
  GemmLowpScope lowp(a.lowp_iter2);
  double* G = ar.dalloc((size_t)B * nn);
  {
    GemmBatch g;
    g.batch = B;
    g.transA = 1; g.transB = 0;
    g.m = n; g.n = n; g.k = n;
    g.A = Y1; g.lda = n; g.sA = nn;
    g.B = Y1; g.ldb = n; g.sB = nn;
    g.C = G; g.ldc = n; g.sC = nn;
    g.sym_upper = true;
    dgemm(g, s);
  }
  mirror_upper(B, n, G, n, nn, s);
  Coef8 cc{}, inva{};
  for (int j = 0; j < r; ++j) {
    cc.v[j] = z2.c[2 * j];
    inva.v[j] = 1.0 / z2.a[j];
  }
  double* E = ar.dalloc((size_t)P * nn);
  double* Rc = ar.dalloc((size_t)P * nn);
  double* Ric = ar.dalloc((size_t)P * nn);
  hipLaunchKernelGGL(shift_scale_kernel, grid_for(nn, P), dim3(256), 0, s, n, r, G, E, cc, inva);
  ZCSD_CHECK_LAUNCH();
  chol_inv_batched(P, n, E, n, nn, Rc, Ric, ar, s);
  double* Ms = G;  // G is dead: reuse for sum_j a_j (G + c_j I)^{-1}
  {
    // one product per term (into Rc, dead after the inversion) and a sum: as
    // one product with inner size r n, the tiles at the top of C would carry
    // r times the work of the average tile and set the launch's length
    GemmBatch g;
    g.batch = P;
    g.transA = 0; g.transB = 1;
    g.m = n; g.n = n; g.k = n;
    g.A = Ric; g.lda = n; g.sA = nn;
    g.B = Ric; g.ldb = n; g.sB = nn;
    g.C = Rc; g.ldc = n; g.sC = nn;
    g.sym_upper = true;
    g.tri = 1 | 8; g.kseg = n;  // R_j^{-1} upper triangular
    dgemm(g, s);
    hipLaunchKernelGGL(sum_terms_upper_kernel, grid_for(nn, B), dim3(256), 0, s, n, r, Rc, Ms);
    ZCSD_CHECK_LAUNCH();
  }
  mirror_upper(B, n, Ms, n, nn, s);
  copy_scale(B, n, n, 1.0, Y1, n, nn, Y2, n, nn, s);
  {
    GemmBatch g;
    g.batch = B;
    g.m = n; g.n = n; g.k = n;
    g.A = Y1; g.lda = n; g.sA = nn;
    g.B = Ms; g.ldb = n; g.sB = nn;
    g.C = Y2; g.ldc = n; g.sC = nn;
    g.alpha = z2.M; g.beta = z2.M;
    dgemm(g, s);
  }
  }  // end of the (possibly FP32) iteration 2
  if (a.lowp_iter2) {
    // Y2 holds the polar factor of R only to the FP32 level; one FP64
    // Newton-Schulz step Y2 <- Y2 + Y2 (I - Y2^T Y2) / 2 restores its
    // orthogonality to the FP64 level (the error left is in the skew part
    // Y2^T Y2 cannot see, of the FP32 products' size)
    GemmFp64Scope fp64;
    ArenaScope ns(ar);
    double* Gn = ar.dalloc((size_t)B * nn);
    double* Tn = ar.dalloc((size_t)B * nn);
    GemmBatch g;
    g.batch = B;
    g.transA = 1;
    g.m = n; g.n = n; g.k = n;
    g.A = Y2; g.lda = n; g.sA = nn;
    g.B = Y2; g.ldb = n; g.sB = nn;
    g.C = Gn; g.ldc = n; g.sC = nn;
    g.sym_upper = true;
    dgemm(g, s);
    mirror_upper(B, n, Gn, n, nn, s);
    GemmBatch h;
    h.batch = B;
    h.m = n; h.n = n; h.k = n;
    h.A = Y2; h.lda = n; h.sA = nn;
    h.B = Gn; h.ldb = n; h.sB = nn;
    h.C = Tn; h.ldc = n; h.sC = nn;
    dgemm(h, s);
    axpby((long long)B * nn, -0.5, Tn, 1.5, Y2, s);
  }

  // 3. W = Q Y2, H = alpha sym(Y2^T R), X1 = Q Y1
  side.join();
  auto qtimes = [&](const double* Y, double* out) {
    GemmBatch g;
    g.batch = B;
    g.m = n; g.n = n; g.k = n;
    g.A = Q; g.lda = n; g.sA = nn;
    g.B = Y; g.ldb = n; g.sB = nn;
    g.C = out; g.ldc = n; g.sC = nn;
    dgemm(g, s);
  };
  qtimes(Y2, a.W);
  if (a.X1) qtimes(Y1, a.X1);
  if (a.H) {
    GemmBatch g;
    g.batch = B;
    g.transA = 1; g.transB = 0;
    g.m = n; g.n = n; g.k = n;
    g.A = Y2; g.lda = n; g.sA = nn;
    g.B = M; g.ldb = n; g.sB = nn;
    g.C = a.H; g.ldc = n; g.sC = nn;
    g.alpha = a.alpha;
    g.tri = 4; g.kseg = n;  // R upper triangular
    dgemm(g, s);
    symmetrize(B, n, a.H, n, nn, s);
  }
  return res;
}

}  // namespace zcsd
