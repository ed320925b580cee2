// Whole CSDs of small full-rank problems, one workgroup per problem, in one
// persistent launch over the batch (Algorithm 1 with Zolo-pd, Sec. 5).
//
// For n <= 64 every matrix of the method fits in LDS, so a problem needs no
// launch sequence and no host decision: one workgroup runs
//   two polars (Zolo-pd, Sec. 5) of A_1 and A_2, each as
//     0. Householder QR  A_i = Q R  (the reflectors stay in LDS);
//        l = 0.9 / ||R^{-1}||_F (floored at eps: a problem whose l reaches
//        eps is reported to the caller, which runs it through the path with
//        Algorithm 2), and the Zolotarev coefficients of the largest
//        tabulated lower bound <= l (a Zolotarev function for a smaller
//        bound still maps [l, 1] into [l_2, 1]);
//     1. QR form on R: for each term, the structured QR of [R; sqrt(c) I],
//        whose reflectors are e_k on top and an upper triangle V2 below, so
//        Q = I - [I; V2] T [I; V2]^T; the first n columns of Q, accumulated
//        backwards from [s I; 0] with s = sqrt(a / sqrt(c)), are two upper
//        triangles Q1, Q2 (Q2 overwrites V2 column by column), and
//        Y1 = M (R + sum_j Q1_j Q2_j^T);
//     2. Cholesky form on Y1: G = Y1^T Y1; for each term the Cholesky factor
//        L_j of (G + c I) / a, its inverse, and Ms += L_j^{-T} L_j^{-1};
//        Y2 = M (Y1 + Y1 Ms);
//     3. H_i = sym(Y2^T R), W_i = Q Y2;
//   B = H_2 - H_1 and its eigenpairs by the Jacobi solve that Zolo-eig uses
//   for blocks of at most 64 (so for n <= 64 Zolo-eig is that solve);
//   U_i = W_i V, theta from the diagonals of V^T H_i V (Algorithm 1,
//   Remark (iii)) or from the eigenvalues (Remark (iv)), sorted ascending.
// The same arithmetic as the class path, in another order: rounding differs.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "jacobi_block.h"
#include "zcsd_internal.h"
#include "zcsd_zolo.h"

namespace zcsd {

namespace {

constexpr int SN = 64;       // largest problem size
constexpr int SL = SN + 1;   // leading dimension of the LDS matrices
constexpr int ST = 256;      // threads per workgroup
constexpr int SNN = SN * SN; // global scratch matrix stride (doubles)

// One tabulated lower bound and the coefficients of both Zolo-pd steps
// (c_{2j-1} and a_j of the partial fractions, M); all doubles.
struct SmallCoef {
  double ell, r, M1, M2;
  double c1[ZOLO_RMAX], a1[ZOLO_RMAX], c2[ZOLO_RMAX], a2[ZOLO_RMAX];
};
constexpr int kCoefDoubles = (int)(sizeof(SmallCoef) / sizeof(double));

// LDS of the polar phase; matrices column-major: X[col][row]
struct PolarShared {
  double F[SN][SL];   // Householder QR of A_i: R on and above the diagonal, reflectors below
  double Bw[SN][SL];  // structured QR (V2 / Q2 upper, Q1 strictly upper stored transposed); Ms; P
  double Y[SN][SL];   // Y1
  double D[SN][SL];   // R^{-1}; G (upper) with L_j (strictly lower, diagonal in dg); Y2 / W
  double tau0[SN], tau[SN], q1d[SN], dg[SN], vb[2][SN], xb[SN];
};

// LDS of the angle and output phase
struct OutShared {
  double V[SN][SL];   // eigenvectors, V[col][row]
  double Ha[SN][SL];  // H_1, then W_1 / W_2
  double Hb[SN][SL];  // H_2
};

struct SmallShared {
  union {
    PolarShared p;
    JacobiShared j;
    OutShared o;
  } u;
  SmallCoef coef;
  double red[ST / 64];
  double lam[SN];
  double th[SN];
  int rank[SN];
  int flag;
};

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum over the four lanes 4g .. 4g+3 of a wave
__device__ inline double quad_sum(double v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  return v;
}

// sum of v over the workgroup (every thread gets it)
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < ST / 64; ++q) t += red[q];
  return t;
}

// One polar of the n x n block A (ld n): writes H (n x n, ld n) and W (n x n,
// ld n) to global memory.  Returns 0, 1 (l reached eps) or 2 (a Cholesky
// factorization broke down); every thread returns the same value.
__device__ int small_polar(int n, const double* __restrict__ A, const SmallCoef* __restrict__ table,
                           int ntab, double eps, double* Hout, double* Wout, SmallShared& sh,
                           int* r_used) {
  PolarShared& P = sh.u.p;
  const int tid = threadIdx.x;
  const int g = tid >> 2, p = tid & 3;  // four threads per column (or row) g
  for (int e = tid; e < n * n; e += ST) P.F[e / n][e % n] = A[e];
  __syncthreads();

  // 0. Householder QR of F
  for (int k = 0; k < n; ++k) {
    if (tid < 64) {
      const int i = tid;
      const double x = (i > k && i < n) ? P.F[k][i] : 0.0;
      const double s2 = wave_sum(x * x);
      const double x0 = P.F[k][k];
      double tau = 0.0, scale = 0.0, beta = x0;
      if (s2 > 0.0) {
        beta = -copysign(sqrt(x0 * x0 + s2), x0);
        tau = (beta - x0) / beta;
        scale = 1.0 / (x0 - beta);
      }
      if (i > k && i < n) P.F[k][i] = x * scale;
      if (i == 0) {
        P.tau0[k] = tau;
        P.F[k][k] = beta;
      }
    }
    __syncthreads();
    const double tk = P.tau0[k];
    if (g > k && g < n && tk != 0.0) {
      double w = 0.0;
      for (int i = k + ((p - k) & 3); i < n; i += 4) w += (i == k ? 1.0 : P.F[k][i]) * P.F[g][i];
      w = quad_sum(w) * tk;
      for (int i = k + ((p - k) & 3); i < n; i += 4) P.F[g][i] -= w * (i == k ? 1.0 : P.F[k][i]);
    }
    __syncthreads();
  }

  // l from ||R^{-1}||_F: R^{-1} into D column by column (D[j][i] = (R^{-1})_ij)
  for (int j = 0; j < n; ++j) {
    double x = 0.0;
    if (tid < j) {
      for (int m = tid; m < j; ++m) x += P.D[m][tid] * P.F[j][m];
    }
    const double dj = 1.0 / P.F[j][j];
    __syncthreads();
    if (tid < j) P.D[j][tid] = -dj * x;
    if (tid == j) P.D[j][j] = dj;
    __syncthreads();
  }
  double ss = 0.0;
  for (int e = tid; e < n * n; e += ST) {
    const int i = e % n, j = e / n;
    if (i <= j) ss += P.D[j][i] * P.D[j][i];
  }
  ss = block_sum(ss, sh.red);
  double ell = (isfinite(ss) && ss > 0.0) ? 0.9 / sqrt(ss) : 0.0;
  ell = fmin(1.0, fmax(ell, eps));
  if (ell <= eps * (1.0 + 1e-12)) return 1;  // uniform: every thread has the same ss
  // the largest tabulated bound <= l (the table descends; its last entry is eps)
  int t = ntab - 1;
  for (int q = 0; q < ntab; ++q)
    if (table[q].ell <= ell) {
      t = q;
      break;
    }
  {
    const double* src = reinterpret_cast<const double*>(table + t);
    double* dst = reinterpret_cast<double*>(&sh.coef);
    for (int e = tid; e < kCoefDoubles; e += ST) dst[e] = src[e];
  }
  __syncthreads();
  const int r = (int)sh.coef.r;
  *r_used = r;

  // 1. QR form on R
  for (int e = tid; e < n * n; e += ST) P.Y[e / n][e % n] = 0.0;
  for (int j = 0; j < r; ++j) {
    const double d = sqrt(sh.coef.c1[j]);
    const double sc = sqrt(sh.coef.a1[j] / d);
    for (int e = tid; e < n * n; e += ST) {
      const int i = e % n, c = e / n;
      if (i <= c) P.Bw[c][i] = (i == c) ? d : 0.0;
    }
    __syncthreads();
    // forward: the reflector of column k acts on top row k and bottom rows 0..k
    for (int k = 0; k < n; ++k) {
      if (tid < 64) {
        const int i = tid;
        const double x = (i <= k) ? P.Bw[k][i] : 0.0;
        const double s2 = wave_sum(x * x);  // >= d^2 > 0: row k of the bottom is still d
        const double x0 = P.F[k][k];
        const double beta = -copysign(sqrt(x0 * x0 + s2), x0);
        if (i <= k) P.Bw[k][i] = x / (x0 - beta);
        if (i == 0) P.tau[k] = (beta - x0) / beta;
      }
      __syncthreads();
      if (g > k && g < n) {
        const double tk = P.tau[k];
        double w = 0.0;
        for (int i = p; i <= k; i += 4) w += P.Bw[k][i] * P.Bw[g][i];
        w = (quad_sum(w) + P.F[g][k]) * tk;  // top row k of column g is still R(k, g)
        for (int i = p; i <= k; i += 4) P.Bw[g][i] -= w * P.Bw[k][i];
      }
      __syncthreads();
    }
    // backward: the first n columns of Q from [sc I; 0]; Q2 overwrites V2,
    // Q1 (k, c) for k < c goes to Bw[k][c], its diagonal to q1d
    if (tid < 64 && tid <= n - 1) P.vb[(n - 1) & 1][tid] = P.Bw[n - 1][tid];
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
      const double* v = P.vb[k & 1];
      const double tk = P.tau[k];
      if (g == k - 1) {
        for (int i = p; i <= k - 1; i += 4) P.vb[(k - 1) & 1][i] = P.Bw[k - 1][i];
      } else if (g == k) {
        for (int i = p; i <= k; i += 4) P.Bw[k][i] = -tk * sc * v[i];
        if (p == 0) P.q1d[k] = sc - tk * sc;
      } else if (g > k && g < n) {
        double w = 0.0;
        for (int i = p; i <= k; i += 4) w += v[i] * P.Bw[g][i];
        w = quad_sum(w) * tk;
        for (int i = p; i <= k; i += 4) P.Bw[g][i] -= w * v[i];
        if (p == 0) P.Bw[k][g] = -w;
      }
      __syncthreads();
    }
    // Y += Q1 Q2^T: (i, l) sums over m >= max(i, l)
    for (int e = tid; e < n * n; e += ST) {
      const int i = e % n, l = e / n;
      double acc = 0.0;
      for (int m = max(i, l); m < n; ++m) {
        const double q1 = (m == i) ? P.q1d[m] : P.Bw[i][m];
        acc += q1 * P.Bw[m][l];
      }
      P.Y[l][i] += acc;
    }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += ST) {
    const int i = e % n, l = e / n;
    P.Y[l][i] = sh.coef.M1 * (P.Y[l][i] + (i <= l ? P.F[l][i] : 0.0));
  }
  __syncthreads();

  // 2. Cholesky form on Y1: G (upper) in D, Ms in Bw
  for (int e = tid; e < n * n; e += ST) {
    const int i = e % n, l = e / n;
    if (i <= l) {
      double acc = 0.0;
      for (int m = 0; m < n; ++m) acc += P.Y[i][m] * P.Y[l][m];
      P.D[l][i] = acc;
    }
    P.Bw[l][i] = 0.0;
  }
  __syncthreads();
  int status = 0;
  for (int j = 0; j < r; ++j) {
    const double c = sh.coef.c2[j], inva = 1.0 / sh.coef.a2[j];
    // L L^T = (G + c I) / a, L(i, k) for i > k in D[k][i], L(k, k) in dg[k]
    for (int k = 0; k < n; ++k) {
      if (tid < 64) {
        const int i = tid;
        double s = 0.0;
        if (i == k)
          for (int m = 0; m < k; ++m) s += P.D[m][k] * P.D[m][k];
        if (i == k) {
          const double dkk = (P.D[k][k] + c) * inva - s;
          if (!(dkk > 0.0)) sh.flag = 2;
          P.dg[k] = sqrt(fmax(dkk, 0x1p-1022));
        }
      }
      __syncthreads();
      if (g > k && g < n) {
        double s = 0.0;
        for (int m = p; m < k; m += 4) s += P.D[m][g] * P.D[m][k];
        s = quad_sum(s);
        if (p == 0) P.D[k][g] = (P.D[g][k] * inva - s) / P.dg[k];
      }
      __syncthreads();
    }
    // L^{-1} in place (last column first)
    for (int jj = n - 1; jj >= 0; --jj) {
      const double dinv = 1.0 / P.dg[jj];
      if (g > jj && g < n) {
        double x = 0.0;
        for (int m = jj + 1 + p; m <= g; m += 4) x += ((m == g) ? P.dg[g] : P.D[m][g]) * P.D[jj][m];
        x = quad_sum(x);
        if (p == 0) P.xb[g] = -dinv * x;
      }
      __syncthreads();
      if (g > jj && g < n && p == 0) P.D[jj][g] = P.xb[g];
      if (tid == 0) P.dg[jj] = dinv;
      __syncthreads();
    }
    // Ms += L^{-T} L^{-1}: (i, l) sums over m >= max(i, l)
    for (int e = tid; e < n * n; e += ST) {
      const int i = e % n, l = e / n;
      double acc = 0.0;
      for (int m = max(i, l); m < n; ++m) {
        const double a = (m == i) ? P.dg[m] : P.D[i][m];
        const double b = (m == l) ? P.dg[m] : P.D[l][m];
        acc += a * b;
      }
      P.Bw[l][i] += acc;
    }
    __syncthreads();
  }
  if (sh.flag == 2) status = 2;
  // Y2 = M (Y1 + Y1 Ms) into D
  for (int e = tid; e < n * n; e += ST) {
    const int i = e % n, l = e / n;
    double acc = 0.0;
    for (int m = 0; m < n; ++m) acc += P.Y[m][i] * P.Bw[l][m];
    P.D[l][i] = sh.coef.M2 * (P.Y[l][i] + acc);
  }
  __syncthreads();

  // 3. H = sym(Y2^T R): P = Y2^T R into Bw, then the symmetric part to global
  for (int e = tid; e < n * n; e += ST) {
    const int i = e % n, l = e / n;
    double acc = 0.0;
    for (int m = 0; m <= l; ++m) acc += P.D[i][m] * P.F[l][m];
    P.Bw[l][i] = acc;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += ST) {
    const int i = e % n, l = e / n;
    Hout[e] = 0.5 * (P.Bw[l][i] + P.Bw[i][l]);
  }
  // W = Q Y2: the reflectors of step 0, last first, on each column of D
  // (four threads per column, each on its own rows: no barrier inside)
  if (g < n) {
    for (int k = n - 1; k >= 0; --k) {
      const double tk = P.tau0[k];
      if (tk == 0.0) continue;
      double w = 0.0;
      for (int i = k + ((p - k) & 3); i < n; i += 4) w += (i == k ? 1.0 : P.F[k][i]) * P.D[g][i];
      w = quad_sum(w) * tk;
      for (int i = k + ((p - k) & 3); i < n; i += 4) P.D[g][i] -= w * (i == k ? 1.0 : P.F[k][i]);
    }
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += ST) Wout[e] = P.D[e / n][e % n];
  __syncthreads();
  return status;
}

// Persistent kernel: workgroup b solves problems list[b], list[b + grid], ...
// status[t]: 0 done, 1 l reached eps (not written), 2 Cholesky breakdown (not
// written); bits 8.. hold the Zolotarev degree of the two polars (max).
__global__ __launch_bounds__(ST) void csd_small_kernel(
    int count, const int* __restrict__ list, const int* __restrict__ nq, const long long* __restrict__ off,
    const long long* __restrict__ toff, const double* __restrict__ A1, const double* __restrict__ A2,
    double* U1, double* U2, double* V1, double* theta, const SmallCoef* __restrict__ table, int ntab,
    double eps, int theta_from_lambda, double* scratch, int* status) {
  __shared__ SmallShared sh;
  const int tid = threadIdx.x;
  double* Hs1 = scratch + (long long)blockIdx.x * 6 * SNN;
  double* Hs2 = Hs1 + SNN;
  double* Ws1 = Hs2 + SNN;
  double* Ws2 = Ws1 + SNN;
  double* Bs = Ws2 + SNN;
  double* Vs = Bs + SNN;
  for (int t = blockIdx.x; t < count; t += gridDim.x) {
    const int k = list[t];
    const int n = nq[k];
    const long long o = off[k];
    if (tid == 0) sh.flag = 0;
    __syncthreads();
    int r1 = 0, r2 = 0;
    int st = small_polar(n, A1 + o, table, ntab, eps, Hs1, Ws1, sh, &r1);
    if (st == 0) st = small_polar(n, A2 + o, table, ntab, eps, Hs2, Ws2, sh, &r2);
    if (st != 0) {
      if (tid == 0) status[t] = st;
      __syncthreads();
      continue;
    }
    // B = H_2 - H_1 (both exactly symmetric)
    for (int e = tid; e < n * n; e += ST) Bs[e] = Hs2[e] - Hs1[e];
    __syncthreads();
    jacobi_block(n, Bs, n, Vs, n, sh.lam, sh.u.j);
    __syncthreads();
    OutShared& O = sh.u.o;
    for (int e = tid; e < n * n; e += ST) {
      O.V[e / n][e % n] = Vs[e];
      O.Ha[e / n][e % n] = Hs1[e];
      O.Hb[e / n][e % n] = Hs2[e];
    }
    __syncthreads();
    // theta_j from c_j = v_j^T H_1 v_j, s_j = v_j^T H_2 v_j (four threads per column)
    {
      const int j = tid >> 2, p = tid & 3;
      if (j < n) {
        double th;
        if (theta_from_lambda) {
          const double x = fmin(fmax(sh.lam[j], -1.0), 1.0);
          th = 0.7853981633974483 + asin(x * 0.7071067811865476);
        } else {
          double cj = 0.0, sj = 0.0;
          for (int a = p; a < n; a += 4) {
            double ta = 0.0, tb = 0.0;
            for (int b = 0; b < n; ++b) {
              ta += O.Ha[b][a] * O.V[j][b];
              tb += O.Hb[b][a] * O.V[j][b];
            }
            cj += O.V[j][a] * ta;
            sj += O.V[j][a] * tb;
          }
          cj = quad_sum(cj);
          sj = quad_sum(sj);
          th = atan2(sj, cj);
        }
        if (p == 0) sh.th[j] = fmin(fmax(th, 0.0), 1.5707963267948966);
      }
    }
    __syncthreads();
    if (tid < n) {
      const double tj = sh.th[tid];
      int rk = 0;
      for (int l = 0; l < n; ++l) {
        const double tl = sh.th[l];
        rk += (tl < tj || (tl == tj && l < tid)) ? 1 : 0;
      }
      sh.rank[tid] = rk;
      theta[toff[k] + rk] = tj;
    }
    __syncthreads();
    // V1 and U_i = W_i V, columns in ascending theta
    for (int e = tid; e < n * n; e += ST) {
      const int i = e % n, j = e / n;
      V1[o + i + (long long)sh.rank[j] * n] = O.V[j][i];
      O.Ha[j][i] = Ws1[e];
      O.Hb[j][i] = Ws2[e];
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += ST) {
      const int i = e % n, j = e / n;
      double u1 = 0.0, u2 = 0.0;
      for (int m = 0; m < n; ++m) {
        const double v = O.V[j][m];
        u1 += O.Ha[m][i] * v;
        u2 += O.Hb[m][i] * v;
      }
      const long long dst = o + i + (long long)sh.rank[j] * n;
      U1[dst] = u1;
      U2[dst] = u2;
    }
    if (tid == 0) status[t] = (max(r1, r2) << 8);
    __syncthreads();
  }
}

// the coefficient table for (eps, tol): bounds 0.9 * 10^(-q/8) while above
// eps, then eps itself
const std::vector<SmallCoef>& small_table(double eps, double tol) {
  static std::mutex mu;
  static std::map<std::pair<double, double>, std::vector<SmallCoef>> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({eps, tol});
  if (it != cache.end()) return it->second;
  std::vector<double> bounds;
  for (int q = 0;; ++q) {
    const double l = 0.9 * std::pow(10.0, -q / 8.0);
    if (l <= eps) break;
    bounds.push_back(l);
  }
  bounds.push_back(eps);
  std::vector<SmallCoef> tab;
  for (double l : bounds) {
    int r = zolo_choose_r(l, tol);
    if (r == 0) r = ZOLO_RMAX;
    const ZoloPlan pl = zolo_plan(l, r);
    SmallCoef c{};
    c.ell = l;
    c.r = r;
    c.M1 = pl.step[0].M;
    c.M2 = pl.step[1].M;
    for (int j = 0; j < r; ++j) {
      c.c1[j] = pl.step[0].c[2 * j];
      c.a1[j] = pl.step[0].a[j];
      c.c2[j] = pl.step[1].c[2 * j];
      c.a2[j] = pl.step[1].a[j];
    }
    tab.push_back(c);
  }
  return cache.emplace(std::make_pair(eps, tol), std::move(tab)).first->second;
}

}  // namespace

size_t small_csd_scratch_bytes(int grid) { return (size_t)grid * 6 * SNN * sizeof(double); }

int small_csd_max_n() { return SN; }

void small_csd_launch(int count, const int* d_list, const int* d_n, const long long* d_off,
                      const long long* d_toff, const double* A1, const double* A2, double* U1,
                      double* U2, double* V1, double* theta, double eps, double tol,
                      bool theta_from_lambda, int grid, double* scratch, int* d_status, Arena& ar,
                      hipStream_t s) {
  if (count <= 0) return;
  const std::vector<SmallCoef>& tab = small_table(eps, tol);
  SmallCoef* d_tab = static_cast<SmallCoef*>(ar.alloc(tab.size() * sizeof(SmallCoef)));
  h2d(d_tab, tab.data(), tab.size() * sizeof(SmallCoef), s);
  hipLaunchKernelGGL(csd_small_kernel, dim3(grid), dim3(ST), 0, s, count, d_list, d_n, d_off, d_toff,
                     A1, A2, U1, U2, V1, theta, d_tab, (int)tab.size(), eps, theta_from_lambda ? 1 : 0,
                     scratch, d_status);
  ZCSD_CHECK_LAUNCH();
}

}  // namespace zcsd
