// Whole CSDs of small full-rank problems, one workgroup per problem, in
// persistent launches over the batch, one per tier of sizes (Algorithm 1
// with Zolo-pd, Sec. 5).
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
#include <tuple>
#include <vector>

#include "jacobi_block.h"
#include "zcsd_api_guard.h"
#include "zcsd_internal.h"
#include "zcsd_zolo.h"

namespace zcsd {

namespace {

// Four instances of everything below (SN: largest size, ST: threads of a
// workgroup), tiers of problem sizes: 49..64 with 512 threads (138 KB of
// LDS: one workgroup per compute unit), 33..48 with 256 threads (79 KB: two
// per compute unit), 17..32 with 128 threads (36 KB: four) and at most 16
// with one wave of 64 threads (10 KB: eight); several workgroups per compute
// unit hide each other's latency.  The two largest tiers have two waves per
// SIMD: the column steps use four threads per column and leave the others
// idle, but the Jacobi rounds and the tile products spread over all of them
// and the per-thread arrays shrink (measured at n = 64: 12.7 -> 10.4 ms for
// 512 problems against 256 threads; at n = 40: 6.4 -> 5.7 ms for 1024
// against 192 threads; 17..32 with 256 threads and two workgroups per
// compute unit was slower, 2.6 -> 4.0 ms for 2048 at n = 24).
constexpr int kTiers = 4;
constexpr int kTierMax[kTiers] = {64, 48, 32, 16};
constexpr int kTierPerCu[kTiers] = {1, 2, 4, 8};

// One tabulated lower bound and the coefficients of both Zolo-pd steps
// (c_{2j-1} and a_j of the partial fractions, M); all doubles.
struct SmallCoef {
  double ell, r, M1, M2;
  double c1[ZOLO_RMAX], a1[ZOLO_RMAX], c2[ZOLO_RMAX], a2[ZOLO_RMAX];
};
constexpr int kCoefDoubles = (int)(sizeof(SmallCoef) / sizeof(double));

// LDS of the polar phase; matrices column-major: X[col][row], leading
// dimension SL
template <int SN>
struct PolarShared {
  static constexpr int SL = SN + 1;
  double F[SN][SL];   // Householder QR of A_i: R on and above the diagonal, reflectors below
  double Bw[SN][SL];  // structured QR (V2 / Q2 upper, Q1 strictly upper stored transposed);
                      // then Ms (upper) with (G + c I) / a and L^{-1} (strictly lower); P
  double Y[SN][SL];   // Y1
  double D[SN][SL];   // G (upper) with L (strictly lower); Y2 / W
  double tau0[SN], tau[SN], q1d[SN], dg[SN], ed[SN], xd[SN], vb[2][SN];
};

// LDS of the angle and output phase
template <int SN>
struct OutShared {
  static constexpr int SL = SN + 1;
  double V[SN][SL];   // eigenvectors, V[col][row]
  double Ha[SN][SL];  // H_1, then W_1
  double Hb[SN][SL];  // H_2, then W_2
};

template <int SN, int ST>
struct SmallShared {
  union {
    PolarShared<SN> p;
    JacobiShared<SN, ST> j;
    OutShared<SN> o;
  } u;
  SmallCoef coef;
  double red[ST / 64];
  double lam[SN];
  double th[SN];
  int rank[SN];
  int flag;
};

// v from the lane whose index within its group of four is given by the DPP
// quad permutation CTRL (as two 32-bit moves)
template <int CTRL>
__device__ inline double quad_perm(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// sum over the four lanes 4g .. 4g+3 of a wave (lanes 1,0,3,2 then 2,3,0,1);
// every lane of the group must be active
__device__ inline double quad_sum(double v) {
  v += quad_perm<0xB1>(v);
  v += quad_perm<0x4E>(v);
  return v;
}

// sum of v over the workgroup (every thread gets the same value)
template <int ST>
__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < ST / 64; ++q) t += red[q];
  return t;
}

// Products on n x n LDS operands (n <= SN), SN/16 x 16 SN/ST outputs per
// thread: rows ti + 16 a, columns tl + (ST/16) b (ti = tid % 16, tl = tid /
// 16).  term(i, l, m) is the summand, m runs over [m0(ti, tl), n).
template <int SN, int ST, class Term, class Out>
__device__ inline void tile_product(int n, int m0, Term term, Out out) {
  constexpr int CT = ST / 16, RA = SN / 16, CB = SN / CT;
  const int ti = threadIdx.x & 15, tl = threadIdx.x >> 4;
  double acc[RA][CB] = {};
  for (int m = m0; m < n; ++m) {
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
      for (int b = 0; b < CB; ++b) acc[a][b] += term(ti + 16 * a, tl + CT * b, m);
  }
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int i = ti + 16 * a, l = tl + CT * b;
      if (i < n && l < n) out(i, l, acc[a][b]);
    }
}

// The rows i = p + 4 q (q < SN/4) of a thread p of a group of four: every
// loop over them is unrolled with loads made unconditionally (all LDS
// matrices have SN rows) and masked by a select, so that the loads of a step
// are in flight together; stores are predicated.
#define FOR_ROWS(q, i) _Pragma("unroll") for (int q = 0, i = p; q < SN / 4; ++q, i += 4)

// One polar of the n x n block A (ld n): writes H (n x n, ld n) and W (n x n,
// ld n) to global memory.  Returns 0, 1 (l reached eps) or 2 (a Cholesky
// factorization broke down); every thread returns the same value.  Columns
// (or rows) g are handled by the four threads 4g .. 4g+3, thread p of them
// on the rows i = p (mod 4); a step's reflector is computed by the group of
// its column at the end of the previous step, so a step has one barrier.
template <int SN, int ST>
__device__ int small_polar(int n, const double* __restrict__ A, const SmallCoef* __restrict__ table,
                           int ntab, double eps, double* Hout, double* Wout, SmallShared<SN, ST>& sh,
                           int* r_used) {
  PolarShared<SN>& P = sh.u.p;
  const int tid = threadIdx.x;
  const int g = tid >> 2, p = tid & 3;
  for (int e = tid; e < n * n; e += ST) P.F[e / n][e % n] = A[e];
  __syncthreads();

  // 0. Householder QR of F.  house(c): the reflector of column c from its rows
  // >= c (rows below scaled to v, the diagonal set to beta), by group c
  auto house = [&](int c) {
    double x[SN / 4];
    double s2 = 0.0;
    FOR_ROWS(q, i) {
      x[q] = P.F[c][i];
      s2 += (i > c && i < n) ? x[q] * x[q] : 0.0;
    }
    s2 = quad_sum(s2);
    const double x0 = P.F[c][c];
    double tau = 0.0, scale = 0.0, beta = x0;
    if (s2 > 0.0) {
      beta = -copysign(sqrt(x0 * x0 + s2), x0);
      tau = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    FOR_ROWS(q, i) {
      if (i > c && i < n) P.F[c][i] = x[q] * scale;
      if (i == c) P.F[c][c] = beta;
    }
    if (p == 0) P.tau0[c] = tau;
  };
  if (g == 0) house(0);
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double tk = P.tau0[k];
    if (g > k && g < n) {
      if (tk != 0.0) {
        double v[SN / 4], x[SN / 4];
        double w = 0.0;
        FOR_ROWS(q, i) {
          v[q] = (i == k) ? 1.0 : P.F[k][i];
          x[q] = P.F[g][i];
          w += (i >= k && i < n) ? v[q] * x[q] : 0.0;
        }
        w = quad_sum(w) * tk;
        FOR_ROWS(q, i) {
          if (i >= k && i < n) P.F[g][i] = x[q] - w * v[q];
        }
      }
      if (g == k + 1) house(g);
    }
    __syncthreads();
  }

  // l = 0.9 / ||R^{-1}||_F: column c of R^{-1} by back substitution in group c
  // (x_i kept in D[c][i] by the thread that owns row i; no barrier inside)
  double ss = 0.0;
  if (g < n) {
    const int c = g;
    for (int i = c; i >= 0; --i) {
      double t = 0.0;
      FOR_ROWS(q, m) {
        const double a = P.F[m][i], x = P.D[c][m];
        t += (m > i && m <= c) ? a * x : 0.0;
      }
      t = quad_sum(t);
      const double x = ((i == c ? 1.0 : 0.0) - t) / P.F[i][i];
      if ((i & 3) == p) {
        P.D[c][i] = x;
        ss += x * x;
      }
    }
  }
  ss = block_sum<ST>(ss, sh.red);
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
  for (int e = tid; e < n * n; e += ST) P.Y[e / n][e % n] = 0.0;
  __syncthreads();
  const int r = (int)sh.coef.r;
  *r_used = r;

  // 1. QR form on R
  for (int j = 0; j < r; ++j) {
    const double d = sqrt(sh.coef.c1[j]);
    const double sc = sqrt(sh.coef.a1[j] / d);
    for (int e = tid; e < n * n; e += ST) {
      const int i = e % n, c = e / n;
      if (i <= c) P.Bw[c][i] = (i == c) ? d : 0.0;
    }
    __syncthreads();
    // forward: the reflector of column c acts on top row c and bottom rows
    // 0..c; its bottom part (rows <= c of column c, row c still d > 0)
    // becomes v, computed by group c
    auto shouse = [&](int c) {
      double x[SN / 4];
      double s2 = 0.0;
      FOR_ROWS(q, i) {
        x[q] = P.Bw[c][i];
        s2 += (i <= c) ? x[q] * x[q] : 0.0;
      }
      s2 = quad_sum(s2);
      const double x0 = P.F[c][c];
      const double beta = -copysign(sqrt(x0 * x0 + s2), x0);
      const double scale = 1.0 / (x0 - beta);
      FOR_ROWS(q, i) {
        if (i <= c) P.Bw[c][i] = x[q] * scale;
      }
      if (p == 0) P.tau[c] = (beta - x0) / beta;
    };
    if (g == 0) shouse(0);
    __syncthreads();
    for (int k = 0; k < n; ++k) {
      if (g > k && g < n) {
        const double tk = P.tau[k];
        double v[SN / 4], x[SN / 4];
        double w = 0.0;
        FOR_ROWS(q, i) {
          v[q] = P.Bw[k][i];
          x[q] = P.Bw[g][i];
          w += (i <= k) ? v[q] * x[q] : 0.0;
        }
        w = (quad_sum(w) + P.F[g][k]) * tk;  // top row k of column g is still R(k, g)
        FOR_ROWS(q, i) {
          if (i <= k) P.Bw[g][i] = x[q] - w * v[q];
        }
        if (g == k + 1) shouse(g);
      }
      __syncthreads();
    }
    // backward: the first n columns of Q from [sc I; 0]; Q2 overwrites V2,
    // Q1 (k, c) for k < c goes to Bw[k][c], its diagonal to q1d.  The v of
    // step k is staged by group k at step k + 1 (its column is not touched then)
    if (g == n - 1) {
      FOR_ROWS(q, i) {
        if (i <= n - 1) P.vb[(n - 1) & 1][i] = P.Bw[n - 1][i];
      }
    }
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
      const double* v = P.vb[k & 1];
      const double tk = P.tau[k];
      if (g == k - 1) {
        FOR_ROWS(q, i) {
          if (i <= k - 1) P.vb[(k - 1) & 1][i] = P.Bw[k - 1][i];
        }
      } else if (g == k) {
        FOR_ROWS(q, i) {
          if (i <= k) P.Bw[k][i] = -tk * sc * v[i];
        }
        if (p == 0) P.q1d[k] = sc - tk * sc;
      } else if (g > k && g < n) {
        double vv[SN / 4], x[SN / 4];
        double w = 0.0;
        FOR_ROWS(q, i) {
          vv[q] = v[i];
          x[q] = P.Bw[g][i];
          w += (i <= k) ? vv[q] * x[q] : 0.0;
        }
        w = quad_sum(w) * tk;
        FOR_ROWS(q, i) {
          if (i <= k) P.Bw[g][i] = x[q] - w * vv[q];
        }
        if (p == 0) P.Bw[k][g] = -w;
      }
      __syncthreads();
    }
    // Y += Q1 Q2^T: (i, l) sums Q1(i, m) Q2(l, m) over m >= max(i, l)
    tile_product<SN, ST>(
        n, max(threadIdx.x & 15, threadIdx.x >> 4),
        [&](int i, int l, int m) -> double {
          if (m < i || m < l || i >= n || l >= n) return 0.0;
          const double q1 = (m == i) ? P.q1d[m] : P.Bw[i][m];
          return q1 * P.Bw[m][l];
        },
        [&](int i, int l, double v) { P.Y[l][i] += v; });
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += ST) {
    const int i = e % n, l = e / n;
    P.Y[l][i] = sh.coef.M1 * (P.Y[l][i] + (i <= l ? P.F[l][i] : 0.0));
  }
  __syncthreads();

  // 2. Cholesky form on Y1: G = Y1^T Y1 (upper of D); Ms (upper of Bw)
  tile_product<SN, ST>(
      n, 0,
      [&](int i, int l, int m) -> double {
        return (i <= l && l < n) ? P.Y[i][m] * P.Y[l][m] : 0.0;
      },
      [&](int i, int l, double v) {
        if (i <= l) {
          P.D[l][i] = v;
          P.Bw[l][i] = 0.0;
        }
      });
  __syncthreads();
  int status = 0;
  for (int j = 0; j < r; ++j) {
    const double c = sh.coef.c2[j], inva = 1.0 / sh.coef.a2[j];
    // E = (G + c I) / a: strictly lower part in Bw, diagonal in ed
    for (int e = tid; e < n * n; e += ST) {
      const int i = e % n, l = e / n;
      if (i > l) P.Bw[l][i] = P.D[i][l] * inva;
      if (i == l) P.ed[i] = (P.D[i][i] + c) * inva;
    }
    __syncthreads();
    // right-looking Cholesky E = L L^T: at step k, row g > k of the trailing
    // part loses L(g, k) L(j, k) for k < j <= g (its own j = p mod 4), and
    // L(g, k) goes to D[k][g], L(k, k) to dg[k]
    for (int k = 0; k < n; ++k) {
      const double ekk = P.ed[k];
      if (!(ekk > 0.0) && tid == 0) sh.flag = 2;
      const double dk = sqrt(fmax(ekk, 0x1p-1022));
      if (g > k && g < n) {
        const double rdk = 1.0 / dk;
        const double lg = P.Bw[k][g] * rdk;
        double ek[SN / 4], eg[SN / 4];
        FOR_ROWS(q, jj) {
          ek[q] = P.Bw[k][jj];
          eg[q] = P.Bw[jj][g];
        }
        FOR_ROWS(q, jj) {
          if (jj > k && jj < g) P.Bw[jj][g] = eg[q] - lg * (ek[q] * rdk);
        }
        if ((g & 3) == p) P.ed[g] -= lg * lg;
        if (p == 0) P.D[k][g] = lg;
      }
      if (tid == 0) P.dg[k] = dk;
      __syncthreads();
    }
    // L^{-1}: column c by forward substitution in group c (strictly lower part
    // in Bw, kept by the thread that owns the row; diagonal in xd)
    if (g < n) {
      const int cc = g;
      const double xc = 1.0 / P.dg[cc];
      if (p == 0) P.xd[cc] = xc;
      for (int i = cc + 1; i < n; ++i) {
        double t = 0.0;
        FOR_ROWS(q, m) {
          const double a = P.D[m][i], x = (m == cc) ? xc : P.Bw[cc][m];
          t += (m >= cc && m < i) ? a * x : 0.0;
        }
        t = quad_sum(t);
        if ((i & 3) == p) P.Bw[cc][i] = -t / P.dg[i];
      }
    }
    __syncthreads();
    // Ms += L^{-T} L^{-1} on the upper triangle: (i, l), i <= l, sums over m >= l
    tile_product<SN, ST>(
        n, threadIdx.x >> 4,
        [&](int i, int l, int m) -> double {
          if (i > l || l >= n || m < l) return 0.0;
          const double a = (m == i) ? P.xd[m] : P.Bw[i][m];
          const double b = (m == l) ? P.xd[m] : P.Bw[l][m];
          return a * b;
        },
        [&](int i, int l, double v) {
          if (i <= l) P.Bw[l][i] += v;
        });
    __syncthreads();
  }
  if (sh.flag == 2) status = 2;
  // Y2 = M (Y1 + Y1 Ms) into D (Ms symmetric, its upper triangle stored)
  tile_product<SN, ST>(
      n, 0,
      [&](int i, int l, int m) -> double {
        if (i >= n || l >= n) return 0.0;
        return P.Y[m][i] * (m <= l ? P.Bw[l][m] : P.Bw[m][l]);
      },
      [&](int i, int l, double v) { P.D[l][i] = sh.coef.M2 * (P.Y[l][i] + v); });
  __syncthreads();

  // 3. H = sym(Y2^T R): P = Y2^T R into Bw, then the symmetric part to global
  tile_product<SN, ST>(
      n, 0,
      [&](int i, int l, int m) -> double {
        return (m <= l && i < n && l < n) ? P.D[i][m] * P.F[l][m] : 0.0;
      },
      [&](int i, int l, double v) { P.Bw[l][i] = v; });
  __syncthreads();
  for (int e = tid; e < n * n; e += ST) {
    const int i = e % n, l = e / n;
    Hout[e] = 0.5 * (P.Bw[l][i] + P.Bw[i][l]);
  }
  // W = Q Y2: the reflectors of step 0, last first, on each column of D
  // (four threads per column, each on its own rows: no barrier inside)
  if (g < n) {
    double x[SN / 4];
    FOR_ROWS(q, i) x[q] = P.D[g][i];
    for (int k = n - 1; k >= 0; --k) {
      const double tk = P.tau0[k];
      double v[SN / 4];
      double w = 0.0;
      FOR_ROWS(q, i) {
        v[q] = (i == k) ? 1.0 : P.F[k][i];
        w += (i >= k && i < n) ? v[q] * x[q] : 0.0;
      }
      w = quad_sum(w) * tk;
      FOR_ROWS(q, i) {
        if (i >= k && i < n) x[q] -= w * v[q];
      }
    }
    FOR_ROWS(q, i) {
      if (i < n) P.D[g][i] = x[q];
    }
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += ST) Wout[e] = P.D[e / n][e % n];
  __syncthreads();
  return status;
}

// Persistent kernel: workgroup b solves problems list[b], list[b + grid], ...
// (MINW: waves per SIMD it must allow, which bounds its registers); the list
// length is `count`, or, when drange is not NULL (lists built on the
// device), the list starts at entry drange[0] and has drange[1] entries.
// status[t] (status[list[t]] when st_by_k): 0 done, 1 l reached
// eps (not written), 2 Cholesky breakdown (not written); bits 8.. hold the
// Zolotarev degree of the two polars (max).
template <int SN, int ST, int MINW>
__global__ __launch_bounds__(ST, MINW) void csd_small_kernel(
    int count, const int* __restrict__ drange, const int* __restrict__ list, const int* __restrict__ nq,
    const long long* __restrict__ off, const long long* __restrict__ toff, const double* __restrict__ A1,
    const double* __restrict__ A2, double* U1, double* U2, double* V1, double* theta,
    const SmallCoef* __restrict__ table, int ntab, double eps, int theta_from_lambda, double* scratch,
    int* status, int st_by_k) {
  __shared__ SmallShared<SN, ST> sh;
  constexpr long long SNN = (long long)SN * SN;
  const int tid = threadIdx.x;
  double* Hs1 = scratch + (long long)blockIdx.x * 6 * SNN;
  double* Hs2 = Hs1 + SNN;
  double* Ws1 = Hs2 + SNN;
  double* Ws2 = Ws1 + SNN;
  double* Bs = Ws2 + SNN;
  double* Vs = Bs + SNN;
  int cnt = count;
  if (drange) {
    list += drange[0];
    cnt = drange[1];
  }
  for (int t = blockIdx.x; t < cnt; t += gridDim.x) {
    const int k = list[t];
    const int si = st_by_k ? k : t;
    const int n = nq[k];
    const long long o = off[k];
    if (tid == 0) sh.flag = 0;
    __syncthreads();
    int r1 = 0, r2 = 0;
    int st = small_polar<SN, ST>(n, A1 + o, table, ntab, eps, Hs1, Ws1, sh, &r1);
    if (st == 0) st = small_polar<SN, ST>(n, A2 + o, table, ntab, eps, Hs2, Ws2, sh, &r2);
    if (st != 0) {
      if (tid == 0) status[si] = st;
      __syncthreads();
      continue;
    }
    // B = H_2 - H_1 (both exactly symmetric)
    for (int e = tid; e < n * n; e += ST) Bs[e] = Hs2[e] - Hs1[e];
    __syncthreads();
    jacobi_block(n, Bs, n, Vs, n, sh.lam, sh.u.j);
    __syncthreads();
    OutShared<SN>& O = sh.u.o;
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
    if (tid == 0) status[si] = (max(r1, r2) << 8);
    __syncthreads();
  }
}

// Routing on the device (for the entry point that makes no host decision),
// one workgroup: problems sorted by descending size with a counting sort over
// the sizes 1..64 in LDS (the order within one size is arbitrary; a
// problem's arithmetic does not depend on it), so that each tier's list is a
// contiguous range, largest first, and its workgroups take the big problems
// before the small ones; range[2t], range[2t + 1] = start and length of tier
// t (sizes 49..64, 33..48, 17..32, 1..16).  A size outside 1..64 gets status
// 3 and joins no list.
constexpr int kRouteThreads = 1024;

__global__ __launch_bounds__(kRouteThreads) void small_route_kernel(int batch, const int* __restrict__ nq,
                                                                   int* list, int* range, int* status) {
  __shared__ int bins[65], cur[65];
  const int tid = threadIdx.x;
  if (tid < 65) bins[tid] = 0;
  __syncthreads();
  for (int k = tid; k < batch; k += kRouteThreads) {
    const int n = nq[k];
    if (n < 1 || n > 64) status[k] = 3;
    else atomicAdd(bins + n, 1);
  }
  __syncthreads();
  if (tid == 0) {
    int pos = 0;
    for (int n = 64; n >= 1; --n) {
      cur[n] = pos;
      pos += bins[n];
    }
    for (int t = 0; t < 4; ++t) {
      const int hi = 64 - 16 * t, lo = hi - 15;
      range[2 * t] = cur[hi];
      range[2 * t + 1] = (lo > 1 ? cur[lo - 1] : pos) - cur[hi];
    }
  }
  __syncthreads();
  for (int k = tid; k < batch; k += kRouteThreads) {
    const int n = nq[k];
    if (n >= 1 && n <= 64) list[atomicAdd(cur + n, 1)] = k;
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

int small_csd_tiers(int* max_n, int* per_cu) {
  for (int t = 0; t < kTiers; ++t) {
    if (max_n) max_n[t] = kTierMax[t];
    if (per_cu) per_cu[t] = kTierPerCu[t];
  }
  return kTiers;
}

size_t small_csd_scratch_bytes(const int* grid) {
  size_t e = 0;
  for (int t = 0; t < kTiers; ++t) e += (size_t)grid[t] * kTierMax[t] * kTierMax[t] * 6;
  return e * sizeof(double);
}

void small_csd_launch(const int* tier_count, const int* d_list, const int* d_n, const long long* d_off,
                      const long long* d_toff, const double* A1, const double* A2, double* U1,
                      double* U2, double* V1, double* theta, double eps, double tol,
                      bool theta_from_lambda, const int* grid, double* scratch, int* d_status, Arena& ar,
                      hipStream_t s) {
  int count = 0;
  for (int t = 0; t < kTiers; ++t) count += tier_count[t];
  if (count <= 0) return;
  const std::vector<SmallCoef>& tab = small_table(eps, tol);
  SmallCoef* d_tab = static_cast<SmallCoef*>(ar.alloc(tab.size() * sizeof(SmallCoef)));
  h2d(d_tab, tab.data(), tab.size() * sizeof(SmallCoef), s);
  const int lam = theta_from_lambda ? 1 : 0;
  const int nt = (int)tab.size();
  int first = 0;
  double* scr = scratch;
  for (int t = 0; t < kTiers; ++t) {
    const int c = tier_count[t];
    if (c > 0) {
      const int* li = d_list + first;
      int* stt = d_status + first;
      if (t == 0)
        hipLaunchKernelGGL((csd_small_kernel<64, 512, 1>), dim3(grid[t]), dim3(512), 0, s, c, nullptr, li, d_n,
                           d_off, d_toff, A1, A2, U1, U2, V1, theta, d_tab, nt, eps, lam, scr, stt, 0);
      else if (t == 1)
        hipLaunchKernelGGL((csd_small_kernel<48, 256, 2>), dim3(grid[t]), dim3(256), 0, s, c, nullptr, li, d_n,
                           d_off, d_toff, A1, A2, U1, U2, V1, theta, d_tab, nt, eps, lam, scr, stt, 0);
      else if (t == 2)
        hipLaunchKernelGGL((csd_small_kernel<32, 128, 2>), dim3(grid[t]), dim3(128), 0, s, c, nullptr, li, d_n,
                           d_off, d_toff, A1, A2, U1, U2, V1, theta, d_tab, nt, eps, lam, scr, stt, 0);
      else
        hipLaunchKernelGGL((csd_small_kernel<16, 64, 2>), dim3(grid[t]), dim3(64), 0, s, c, nullptr, li, d_n,
                           d_off, d_toff, A1, A2, U1, U2, V1, theta, d_tab, nt, eps, lam, scr, stt, 0);
      ZCSD_CHECK_LAUNCH();
    }
    first += c;
    scr += (size_t)grid[t] * kTierMax[t] * kTierMax[t] * 6;
  }
}

namespace {

struct DeviceTable {
  const SmallCoef* d;
  int n;
};

// Device copies of the coefficient tables, per (device, eps, tol), made on
// request and kept until the process ends (a few KB each).
std::mutex g_dtab_mu;
std::map<std::tuple<int, double, double>, DeviceTable> g_dtab;

// Workspace of the device-routed launch, in bytes from its start:
// [0, 256) the tier ranges, then the sorted list of `batch` ints, then the
// per-workgroup scratch of the largest tier grid (the tiers run one after
// another on one stream and share it).
size_t dev_lists_bytes(int batch) { return ((size_t)batch * sizeof(int) + 255) / 256 * 256; }

size_t dev_scratch_bytes(int n_cu) {
  size_t e = 0;
  for (int t = 0; t < kTiers; ++t)
    e = std::max(e, (size_t)kTierPerCu[t] * n_cu * kTierMax[t] * kTierMax[t] * 6);
  return e * sizeof(double);
}

}  // namespace

bool small_table_device_make(int device, double eps, double tol) {
  std::lock_guard<std::mutex> lk(g_dtab_mu);
  const auto key = std::make_tuple(device, eps, tol);
  if (g_dtab.count(key)) return false;
  const std::vector<SmallCoef>& tab = small_table(eps, tol);
  void* d = nullptr;
  ZCSD_HIP(hipMalloc(&d, tab.size() * sizeof(SmallCoef)));
  const hipError_t e = hipMemcpy(d, tab.data(), tab.size() * sizeof(SmallCoef), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    ZCSD_HIP(e);
  }
  g_dtab[key] = DeviceTable{static_cast<const SmallCoef*>(d), (int)tab.size()};
  return true;
}

size_t small_device_ws_bytes(int batch, int n_cu) { return 256 + dev_lists_bytes(batch) + dev_scratch_bytes(n_cu); }

void small_device_launch(int device, int batch, const int* d_n, const long long* d_off,
                         const long long* d_toff, const double* A1, const double* A2, double* U1,
                         double* U2, double* V1, double* theta, double eps, double tol,
                         bool theta_from_lambda, int n_cu, void* ws, int* d_status, hipStream_t s) {
  DeviceTable tab{};
  {
    std::lock_guard<std::mutex> lk(g_dtab_mu);
    auto it = g_dtab.find(std::make_tuple(device, eps, tol));
    if (it == g_dtab.end())
      throw ArgError("csd_batched_small: no coefficient table for these eps/tol on this device "
                     "(call zcsd_small_batch_prepare first)");
    tab = it->second;
  }
  char* base = static_cast<char*>(ws);
  int* range = reinterpret_cast<int*>(base);
  int* list = reinterpret_cast<int*>(base + 256);
  double* scr = reinterpret_cast<double*>(base + 256 + dev_lists_bytes(batch));
  hipLaunchKernelGGL(small_route_kernel, dim3(1), dim3(kRouteThreads), 0, s, batch, d_n, list, range,
                     d_status);
  ZCSD_CHECK_LAUNCH();
  const int lam = theta_from_lambda ? 1 : 0;
  for (int t = 0; t < kTiers; ++t) {
    // every tier is launched with its full persistent grid; its workgroups
    // read the range of the list from the device and leave at once if it is short
    const int g = kTierPerCu[t] * n_cu;
    const int* li = list;
    const int* ct = range + 2 * t;
    if (t == 0)
      hipLaunchKernelGGL((csd_small_kernel<64, 512, 1>), dim3(g), dim3(512), 0, s, 0, ct, li, d_n, d_off,
                         d_toff, A1, A2, U1, U2, V1, theta, tab.d, tab.n, eps, lam, scr, d_status, 1);
    else if (t == 1)
      hipLaunchKernelGGL((csd_small_kernel<48, 256, 2>), dim3(g), dim3(256), 0, s, 0, ct, li, d_n, d_off,
                         d_toff, A1, A2, U1, U2, V1, theta, tab.d, tab.n, eps, lam, scr, d_status, 1);
    else if (t == 2)
      hipLaunchKernelGGL((csd_small_kernel<32, 128, 2>), dim3(g), dim3(128), 0, s, 0, ct, li, d_n, d_off,
                         d_toff, A1, A2, U1, U2, V1, theta, tab.d, tab.n, eps, lam, scr, d_status, 1);
    else
      hipLaunchKernelGGL((csd_small_kernel<16, 64, 2>), dim3(g), dim3(64), 0, s, 0, ct, li, d_n, d_off,
                         d_toff, A1, A2, U1, U2, V1, theta, tab.d, tab.n, eps, lam, scr, d_status, 1);
    ZCSD_CHECK_LAUNCH();
  }
}

}  // namespace zcsd

using namespace zcsd;

namespace {

// the options the device-routed entry point takes: FP64, no forced l or r,
// the rank left to the l estimate
zcsd_opts small_batch_opts(const zcsd_opts* opts) {
  zcsd_opts o;
  zcsd_default_opts(&o);
  if (opts) o = *opts;
  ZCSD_REQUIRE(o.prec == ZCSD_FP64, "csd_batched_small: only FP64");
  ZCSD_REQUIRE(o.rank_mode != ZCSD_RANK_DEFICIENT, "csd_batched_small: full-rank problems only");
  ZCSD_REQUIRE(o.r_override == 0 && o.ell_override == 0.0, "csd_batched_small: r and l are not forced here");
  ZCSD_REQUIRE(o.eps > 0.0 && o.eps < 1.0 && o.tol > 0.0, "csd_batched_small: eps/tol out of range");
  ZCSD_REQUIRE(o.postprocess >= 0 && o.postprocess <= 2, "csd_batched_small: postprocess out of range");
  return o;
}

constexpr int kSmallBatchMax = 1 << 20;

int device_cus(int device) {
  int n_cu = 1;
  ZCSD_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device));
  return std::max(n_cu, 1);
}

}  // namespace

extern "C" zcsd_status zcsd_small_batch_prepare(zcsd_handle* handle, int batch, const zcsd_opts* opts,
                                                size_t* ws_bytes) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    ZCSD_REQUIRE(batch >= 1 && batch <= kSmallBatchMax, "csd_batched_small: 1 <= batch <= 2^20");
    ZCSD_REQUIRE(ws_bytes, "csd_batched_small: NULL ws_bytes");
    const zcsd_opts o = small_batch_opts(opts);
    ZCSD_HIP(hipSetDevice(handle->device));
    small_table_device_make(handle->device, o.eps, o.tol);
    *ws_bytes = small_device_ws_bytes(batch, device_cus(handle->device));
  });
}

extern "C" zcsd_status zcsd_dcsd_batched_small(zcsd_handle* handle, int batch, const int* d_n,
                                               const long long* d_off, const long long* d_toff,
                                               const double* d_A1, const double* d_A2, double* d_U1,
                                               double* d_U2, double* d_V1, double* d_theta,
                                               int* d_status, void* d_ws, size_t ws_bytes,
                                               const zcsd_opts* opts) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    ZCSD_REQUIRE(batch >= 1 && batch <= kSmallBatchMax, "csd_batched_small: 1 <= batch <= 2^20");
    ZCSD_REQUIRE(d_n && d_off && d_toff && d_A1 && d_A2 && d_U1 && d_U2 && d_V1 && d_theta && d_status &&
                     d_ws,
                 "csd_batched_small: NULL pointer");
    ZCSD_REQUIRE(((uintptr_t)d_ws & 255) == 0, "csd_batched_small: workspace not 256-byte aligned");
    const zcsd_opts o = small_batch_opts(opts);
    ZCSD_HIP(hipSetDevice(handle->device));
    const int n_cu = device_cus(handle->device);
    ZCSD_REQUIRE(ws_bytes >= small_device_ws_bytes(batch, n_cu),
                 "csd_batched_small: workspace smaller than zcsd_small_batch_prepare's size");
    small_device_launch(handle->device, batch, d_n, d_off, d_toff, d_A1, d_A2, d_U1, d_U2, d_V1, d_theta,
                        o.eps, o.tol, o.postprocess == 2, n_cu, d_ws, d_status, handle->stream);
  });
}
