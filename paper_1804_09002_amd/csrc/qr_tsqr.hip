// Tall panel factorisation for the blocked Householder QR: TSQR followed by
// reconstruction of the Householder vectors.
//
// A panel of h logical rows and w <= 32 columns is cut into P = ceil(h / TS_MB)
// row blocks of TS_MB rows (the last one takes the remainder):
//   A. every block is factored by one workgroup, Q_p R_p (local Householder
//      vectors Y_p and compact-WY factor T_p);
//   B. one workgroup factors the stacked [R_1; ...; R_P] = Q_top R (Q_top is
//      kept as Y_top and Z = T_top Y_top(0:w, :)^T), forms the top w x w block
//      Q_00 of the panel's Q, and the
//      LU factorisation Q_00 - S = L_1 U with the sign of each pivot chosen so
//      that |pivot| >= 1 (S = diag(+-1)).  Then the panel's Householder form is
//      V = [L_1; Q_rest U^{-1}], T = -U S L_1^{-T}, R = S R_tsqr
//      (Ballard, Demmel, Grigori, Jacobsen, Knight, Nguyen, "Reconstructing
//      Householder vectors from tall-skinny QR", 2015);
//   C. every block forms its piece Q_top,p = [I; 0]_p - Y_top,p Z and its rows of
//      the explicit Q, Q_p = (I - Y_p T_p Y_p^T) [Q_top,p; 0], and of V = Q U^{-1}.
// A panel of one block (P = 1), or of up to 512 rows factored by one larger
// workgroup, is finished by stage A alone.
// Each stage is parallel over rows; only the w x w pieces are sequential.
// The Householder factorisations keep the matrix in registers, four columns
// per lane (eight lanes hold a row): a step swizzles the pivot column to the
// eight lanes of each row, every lane forms the dot products with its four
// columns, and a short butterfly plus one sum over the waves gives all 32
// products at once, so a step costs one barrier.  The stacked R
// factors and Y_top are kept row-major, so these loads and stores coalesce.
// The result is interchangeable with a column-by-column Householder panel
// (same R up to row signs, V unit lower trapezoidal, H = I - V T V^T).
#include <algorithm>
#include <cmath>

#include "zcsd_internal.h"
#include "zcsd_la.h"
#include "zcsd_prof.h"
#include "zcsd_qr_tsqr.h"

namespace zcsd {

constexpr int TS_NT = 256;
constexpr int TS_W = 32;  // panel width handled here
constexpr int TS_W1 = TS_W + 1;
constexpr int TS_LOCAL_RQ = TS_MB / (8 * (TS_NT / 64));  // row slots per lane, local
constexpr int TS_TREE_NT = 512;                           // tree workgroup
constexpr int TS_TREE_RQ = (TS_PMAX * TS_W + TS_TREE_NT / 8 - 1) / (TS_TREE_NT / 8);  // tree

__device__ __forceinline__ int ts_phys(int i, int h1, int r1a, int r2a) {
  return i < h1 ? r1a + i : r2a + (i - h1);
}
// logical row -> row of V (the second segment may start at row vr2 of V)
__device__ __forceinline__ int ts_vrow(int i, int h1, int vr2) { return i < h1 ? i : vr2 + (i - h1); }

// Cross-lane moves of doubles (two 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// ds_swizzle in bit mode on both halves of a double: lane l (within its 32-lane
// half) reads lane ((l & AND) | OR) ^ XOR
template <int AND, int OR, int XOR>
__device__ __forceinline__ double swizzle_f64(double v) {
  constexpr int pat = AND | (OR << 5) | (XOR << 10);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)b, pat);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), pat);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// (a, b) -> a' + b' after swapping the upper half-wave of a with the lower
// half-wave of b (P32), or the odd 16-lane rows of a with the even rows of b:
// a lane of the lower half ends with a + partner's a, one of the upper half
// with partner's b + b -- one halving step of the butterfly below.
template <bool P32>
__device__ __forceinline__ double swap_sum(double a, double b) {
  const long long ia = __double_as_longlong(a), ib = __double_as_longlong(b);
  const unsigned alo = (unsigned)ia, ahi = (unsigned)(ia >> 32);
  const unsigned blo = (unsigned)ib, bhi = (unsigned)(ib >> 32);
  unsigned a0, b0, a1, b1;
  if constexpr (P32) {
    const auto rl = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    a0 = rl[0]; b0 = rl[1]; a1 = rh[0]; b1 = rh[1];
  } else {
    const auto rl = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    a0 = rl[0]; b0 = rl[1]; a1 = rh[0]; b1 = rh[1];
  }
  return __longlong_as_double(((long long)a1 << 32) | a0) +
         __longlong_as_double(((long long)b1 << 32) | b0);
}

typedef double d4 __attribute__((ext_vector_type(4)));

// 16 x 16 tile (ti, tj) of C = X Y with K = KD on the FP64 matrix cores;
// fx(i, k) and fy(k, j) read the operands (LDS or global).  v_mfma_f64_16x16x4f64
// takes a[i][k] from lane i + 16k and b[k][j] from lane j + 16k and leaves
// d[i][j] in item i / 4 of lane j + 16 (i % 4); fed with Y^T as "a" and X^T as
// "b" it holds the transposed tile, so item v of lane l is
// C[16 ti + l % 16][16 tj + 4 v + l / 16] (tile_row / tile_col below).
template <int KD, class FX, class FY>
__device__ __forceinline__ d4 mfma_tile(FX fx, FY fy, int ti, int tj) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < KD; kk += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fy(kk + lk, 16 * tj + lr), fx(16 * ti + lr, kk + lk),
                                               acc, 0, 0, 0);
  return acc;
}
__device__ __forceinline__ int tile_row(int ti) { return 16 * ti + (threadIdx.x & 15); }
__device__ __forceinline__ int tile_col(int tj, int v) { return 16 * tj + 4 * v + ((threadIdx.x & 63) >> 4); }

// Inverse of the upper-triangular 32 x 32 A (LDS, exact zeros below the
// diagonal, identity beyond the active size) into I, for two matrices at once
// (m = 0, 1; A1 may be null): the 16 x 16 diagonal blocks by back
// substitution, one column per thread (threads 0..63), then (I)_AB = -I_A
// (A_AB I_B) as two 16 x 16 MFMA products (wave m); X (32 x 32) is scratch.
// Three barriers.
__device__ void lds_upper_inverse32x2(const double (*A0)[TS_W1], double (*I0)[TS_W1],
                                      const double (*A1)[TS_W1], double (*I1)[TS_W1],
                                      double (*X)[TS_W1]) {
  const int tid = threadIdx.x, wave = tid >> 6;
  const int nm = A1 ? 2 : 1;
  if (tid < 32 * nm) {
    const int m = tid >> 5, o = tid & 16, c = tid & 15;
    const double (*A)[TS_W1] = m ? A1 : A0;
    double (*I)[TS_W1] = m ? I1 : I0;
    double x[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double sacc = 0.0;
#pragma unroll
      for (int q = i + 1; q < 16; ++q) sacc = fma(A[o + i][o + q], x[q], sacc);
      x[i] = (i > c) ? 0.0 : (((i == c) ? 1.0 : -sacc) / A[o + i][o + i]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) I[o + i][o + c] = x[i];
  } else if (tid >= 64 && tid < 64 + 32 * nm) {  // the blocks below the diagonal
    const int m = (tid >> 5) & 1, c = tid & 15, r0 = tid & 16;
    double (*I)[TS_W1] = m ? I1 : I0;
#pragma unroll
    for (int i = 0; i < 8; ++i) I[16 + (r0 >> 1) + i][c] = 0.0;
  }
  __syncthreads();
  if (wave < nm) {
    const double (*A)[TS_W1] = wave ? A1 : A0;
    double (*I)[TS_W1] = wave ? I1 : I0;
    const d4 t = mfma_tile<16>([&](int i, int k) { return A[i][16 + k]; },
                               [&](int k, int j) { return I[16 + k][16 + j]; }, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) X[16 * wave + tile_row(0)][tile_col(0, v)] = t[v];
  }
  __syncthreads();
  if (wave < nm) {
    double (*I)[TS_W1] = wave ? I1 : I0;
    const d4 t = mfma_tile<16>([&](int i, int k) { return I[i][k]; },
                               [&](int k, int j) { return X[16 * wave + k][j]; }, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) I[tile_row(0)][16 + tile_col(0, v)] = -t[v];
  }
  __syncthreads();
}

// Householder QR of a rows x w matrix (w <= 32) held in registers, four
// columns per lane: lane l of wave v holds columns 4g .. 4g + 3 (g = l % 8) on
// the rows i = 8 RQ v + 8 r + h (h = l / 8), r < RQ, in a[r][0..3] (zeros
// beyond rows and w).
// Step t sends the pivot column to the eight lanes of each row set with one
// swizzle (its rows above t zeroed); every lane forms the partial dot products
// of the pivot column with its four columns; a butterfly over the eight row
// sets of the wave (lane ^ 32, ^ 16, ^ 8) leaves one column's wave sum per
// lane, the waves are summed through LDS (one barrier) and each lane gathers
// the totals of its four columns: d_j = sum_{i >= t} a_it a_ij for every j at
// once.  With alpha = a_tt, beta = -sign(alpha) sqrt(d_t), tau = (beta -
// alpha) / beta and scal = 1 / (alpha - beta), the reflector is
// v = scal (a_t - beta e_t) and v^T a_j = scal (d_j - beta a_tj), so columns
// j > t are updated in place with their own coefficients.  Column t is left
// unscaled: the lane keeps scal_t and beta_t, and the vector is
// y_t = scal_t a_t below the diagonal (products with it carry a factor
// scal_t).  The same sums give column t of the strictly upper part of Y^T Y
// (y_k^T v, k < t), kept with tau_t for T after the loop.
// On return, for a lane column j: rows i < j hold R(i, j), R(j, j) = beta_j,
// rows i > j hold Y(i, j) / scal_j.
// NW (4 or 8) waves of 64 lanes.  LDS: red[2 * NW * 32], rowb[2 * 32],
// Zm[32][33], taus[32].
template <int t, int RQ, int NW>
__device__ __forceinline__ void ql_householder_step(double (&a)[RQ][4], double (&myscal)[4],
                                                    double (&mybeta)[4], double (*Zm)[TS_W1],
                                                    double* taus, double* red, double* rowb) {
  static_assert(NW == 4 || NW == 8, "4 or 8 waves");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane & 7, h = lane >> 3;
  constexpr int gt = t >> 2, qt = t & 3;  // the lanes g == gt hold column t in slot qt
  constexpr int rt = t >> 3, ht = t & 7;  // row t: wave 0, slot rt, row set ht
  constexpr int buf = t & 1;
  // pivot column, from lane (h, gt) to the lanes (h, *); rows above t zeroed
  double colt[RQ];
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    const double c = swizzle_f64<0x18, gt, 0>(a[r][qt]);
    colt[r] = (8 * r < t && wave == 0 && 8 * r + h < t) ? 0.0 : c;
  }
  double p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < RQ; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = fma(colt[r], a[r][q], p[q]);
  // sum over the row sets: lane ^ 32 keeps q in {0,1} / {2,3}, lane ^ 16 keeps
  // one q, lane ^ 8 adds the last pair: lane holds column 4g + ((lane >> 4) & 3)
  const double x0 = swap_sum<true>(p[0], p[2]);
  const double x1 = swap_sum<true>(p[1], p[3]);
  double y = swap_sum<false>(x0, x1);
  y += dpp_f64<0x128>(y);  // row_ror:8
  double* rb = red + buf * NW * TS_W;
  double* pr = rowb + buf * TS_W;
  const int jsel = 4 * g + ((lane >> 4) & 3);
  if ((lane & 8) == 0) rb[wave * TS_W + jsel] = y;
  if (wave == 0 && h == ht) {
#pragma unroll
    for (int q = 0; q < 4; ++q) pr[4 * g + q] = a[rt][q];  // the pivot row a(t, :)
  }
  __syncthreads();
  // the totals of the lane's own four columns, read straight from the waves'
  // partial sums (one LDS round trip; pairwise sums in a fixed order)
  double d[4], at[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double* c = rb + 4 * g + q;
    double v = (c[0] + c[TS_W]) + (c[2 * TS_W] + c[3 * TS_W]);
    if constexpr (NW == 8) v += (c[4 * TS_W] + c[5 * TS_W]) + (c[6 * TS_W] + c[7 * TS_W]);
    d[q] = v;
    at[q] = pr[4 * g + q];
  }
  const double dt = readlane_f64(d[qt], gt), alpha = readlane_f64(at[qt], gt);
  double tau = 0.0, beta = 0.0, scal = 0.0;
  if (dt > 0.0) {
    const double nrm = sqrt(dt);
    beta = alpha >= 0.0 ? -nrm : nrm;
    tau = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
  if (g == gt) {
    myscal[qt] = scal;
    mybeta[qt] = beta;
  }
  // w_q = v^T a_j (j > t) or (y_j^T v) / scal_j (j < t), j = 4g + q
  double coef[4], c2[4], wq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    wq[q] = scal * (d[q] - beta * at[q]);
    coef[q] = (4 * g + q > t) ? tau * wq[q] : 0.0;
    c2[q] = coef[q] * scal;
  }
  // a_j -= tau v (v^T a_j), j > t; v = scal * pivot column below row t, 1 on row t
  const bool onrow = (wave == 0 && h == ht);
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    if (r == rt) {
      const double vr = onrow ? 1.0 : scal * colt[r];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[r][q] = fma(-coef[q], vr, a[r][q]);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) a[r][q] = fma(-c2[q], colt[r], a[r][q]);
    }
  }
  // strictly upper Y^T Y (column t: y_k^T v = scal_k w, k < t) and tau
  if (tid < 8) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (4 * g + q < t) Zm[4 * g + q][t] = myscal[q] * wq[q];
    if (g == gt) taus[t] = tau;
  }
}

// the 32 steps, unrolled at compile time so that every register index is static
template <int t, int RQ, int NW>
__device__ __forceinline__ void ql_householder_steps(double (&a)[RQ][4], int w, double (&myscal)[4],
                                                     double (&mybeta)[4], double (*Zm)[TS_W1],
                                                     double* taus, double* red, double* rowb) {
  if constexpr (t < TS_W) {
    if (t < w) {
      ql_householder_step<t, RQ, NW>(a, myscal, mybeta, Zm, taus, red, rowb);
      ql_householder_steps<t + 1, RQ, NW>(a, w, myscal, mybeta, Zm, taus, red, rowb);
    }
  }
}

// The factorisation, then T from the UT relation T^{-1} = striu(Y^T Y) +
// diag(1 / tau) (for H = I - Y T Y^T with T upper triangular), inverted by
// 16 x 16 blocks on the matrix cores.  A step with tau = 0 (a zero column, H =
// I) is decoupled: its row and column of T are zero.  Ts receives T; Zm and X
// (32 x 33 each) and taus[32] are scratch.  Ends with a barrier.
template <int RQ, int NW>
__device__ void ql_householder(double (&a)[RQ][4], int w, double (&myscal)[4], double (&mybeta)[4],
                               double (*Ts)[TS_W1], double (*Zm)[TS_W1], double (*X)[TS_W1],
                               double* taus, double* red, double* rowb) {
  if (threadIdx.x < TS_W) taus[threadIdx.x] = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    myscal[q] = 0.0;
    mybeta[q] = 0.0;
  }
  __syncthreads();
  ql_householder_steps<0, RQ, NW>(a, w, myscal, mybeta, Zm, taus, red, rowb);
  __syncthreads();
  for (int e = threadIdx.x; e < TS_W * TS_W; e += 64 * NW) {
    const int i = e & (TS_W - 1), jj = e / TS_W;
    const double ti = taus[i], tj = taus[jj];
    double v = 0.0;
    if (i < jj) v = (ti != 0.0 && tj != 0.0) ? Zm[i][jj] : 0.0;
    else if (i == jj) v = (ti != 0.0) ? 1.0 / ti : 1.0;
    Zm[i][jj] = v;
  }
  __syncthreads();
  lds_upper_inverse32x2(Zm, Ts, nullptr, nullptr, X);
  if (threadIdx.x < TS_W && taus[threadIdx.x] == 0.0) Ts[threadIdx.x][threadIdx.x] = 0.0;
  __syncthreads();
}

// R(i, j) and Y(i, j) of a lane column j on logical row i (see above)
__device__ __forceinline__ double cl_rval(double v, int i, int j, double mybeta) {
  return (i < j) ? v : ((i == j) ? mybeta : 0.0);
}
__device__ __forceinline__ double cl_yval(double v, int i, int j, double myscal) {
  return (i < j) ? 0.0 : ((i == j) ? 1.0 : myscal * v);
}
// ---------------------------------------------------------------------------
// A: local QR of every row block
// With direct != 0 (a panel of one block, P = 1) the block's Householder QR is
// the panel's: R goes into the matrix (zeros below it), Y into V and T into
// Tfin, and the tree and expansion stages are not needed.
// NW waves hold 64 NW rows (eight row slots per lane); NW = 8 serves direct
// panels of up to 512 rows.
template <int NW>
__global__ __launch_bounds__(64 * NW) void tsqr_local_kernel(
    double* M, long long ldm, long long sM, int c0, int w, int h1, int r1a, int r2a, int h,
    int P, double* V, long long ldv, long long sV, int vr2, double* Tloc, double* Rstack,
    long long sScr, int direct, double* Tfin, long long sT) {
  constexpr int NT = 64 * NW, MBK = 8 * TS_LOCAL_RQ * NW;  // threads, rows per block
  __shared__ double red[2 * NW * TS_W], rowb[2 * TS_W], taus[TS_W];
  __shared__ double Ts[TS_W][TS_W1];
  __shared__ double Zm[TS_W][TS_W1];
  __shared__ double Xs[TS_W][TS_W1];
  const int p = blockIdx.x;
  const long long b = blockIdx.y;
  M += b * sM;
  V += b * sV;
  const int i0 = p * MBK;
  const int rows = min(MBK, h - i0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane & 7, hs = lane >> 3;
  double a[TS_LOCAL_RQ][4];
#pragma unroll
  for (int r = 0; r < TS_LOCAL_RQ; ++r) {
    const int i = 8 * TS_LOCAL_RQ * wave + 8 * r + hs;
    const long long pr = (i < rows) ? ts_phys(i0 + i, h1, r1a, r2a) : 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = 4 * g + q;
      a[r][q] = (i < rows && j < w) ? M[pr + (long long)(c0 + j) * ldm] : 0.0;
    }
  }
  double myscal[4], mybeta[4];
  ql_householder<TS_LOCAL_RQ, NW>(a, w, myscal, mybeta, Ts, Zm, Xs, taus, red, rowb);
  // R_p (rows 0..31 of the block, row-major, zero beyond the block and w) and
  // Y_p (unit lower trapezoidal) into V's rows, straight from the lanes
  double* Rp = Rstack + b * sScr;
#pragma unroll
  for (int r = 0; r < TS_LOCAL_RQ; ++r) {
    const int i = 8 * TS_LOCAL_RQ * wave + 8 * r + hs;
    const long long vi = (i < rows) ? ts_vrow(i0 + i, h1, vr2) : 0;
    const long long pr = (i < rows) ? ts_phys(i0 + i, h1, r1a, r2a) : 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = 4 * g + q;
      if (direct) {
        if (i < rows && j < w) M[pr + (long long)(c0 + j) * ldm] = cl_rval(a[r][q], i, j, mybeta[q]);
      } else if (8 * r < TS_W && wave == 0 && i < w) {
        Rp[(p * w + i) * TS_W + j] = (j < w && i < rows) ? cl_rval(a[r][q], i, j, mybeta[q]) : 0.0;
      }
      if (i < rows && j < w) V[vi + (long long)j * ldv] = cl_yval(a[r][q], i, j, myscal[q]);
    }
  }
  double* Tp = direct ? Tfin + b * sT : Tloc + b * sScr + (long long)p * TS_W * TS_W;
  for (int e = tid; e < TS_W * TS_W; e += NT) Tp[e] = Ts[e % TS_W][e / TS_W];
}

// B: QR of the stacked R factors (registers), explicit Q_top, reconstruction
// pieces (w x w work in LDS).
template <int RQ>
__global__ __launch_bounds__(TS_TREE_NT) void tsqr_tree_kernel(
    double* M, long long ldm, long long sM, int c0, int w, int h1, int r1a, int r2a, int P,
    const double* V, long long ldv, long long sV, int vr2, const double* Tloc, const double* Rstack,
    double* Qtop, double* Zo, double* Uo, double* Lo, double* So, long long sScr, double* Tfin,
    long long sT) {
  constexpr int NWT = TS_TREE_NT / 64;
  static_assert(RQ >= 4, "wave 0 must hold the first 32 stacked rows");
  __shared__ double red[2 * NWT * TS_W], rowb[2 * TS_W], taus[TS_W];
  __shared__ double Ts[TS_W][TS_W1];  // T_top
  __shared__ double Yt[TS_W][TS_W1];  // Y_top(0:w, 0:w), then X2
  __shared__ double Z[TS_W][TS_W1];   // T_top Y_top(0:w, :)^T, then L1^{-T}
  __shared__ double Rf[TS_W][TS_W1];  // R_tsqr
  __shared__ double Q0[TS_W][TS_W1];  // Q_top,0, then Q_00 and its LU
  __shared__ double Y0[TS_W][TS_W1];  // Y_0(0:w, 0:w) of block 0
  __shared__ double T0s[TS_W][TS_W1]; // T_0 of block 0, then U
  __shared__ double sg[TS_W], pv[TS_W];
  const long long b = blockIdx.x;
  M += b * sM;
  V += b * sV;
  Tloc += b * sScr;
  Rstack += b * sScr;
  Qtop += b * sScr;
  Zo += b * sScr;
  Uo += b * sScr;
  Lo += b * sScr;
  So += b * sScr;
  Tfin += b * sT;
  const int tid = threadIdx.x;
  const int rows = P * w;
  {
    const int lane = tid & 63, wv = tid >> 6;
    const int g = lane & 7, hs = lane >> 3;
    double a[RQ][4];
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
      const int i = 8 * RQ * wv + 8 * r + hs;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = 4 * g + q;
        a[r][q] = (i < rows && j < w) ? Rstack[i * TS_W + j] : 0.0;
      }
    }
    double myscal[4], mybeta[4];
    ql_householder<RQ, NWT>(a, w, myscal, mybeta, Ts, Z, Q0, taus, red, rowb);
    // Y_top (unit lower trapezoidal, explicit, row-major) to global memory:
    // every expansion block forms its own rows of Q_top = [I; 0] - Y_top Z.
    // R_tsqr and Y_top(0:w, 0:w) from the first w rows (rows w..31 belong to
    // the next block: zero here).
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
      const int i = 8 * RQ * wv + 8 * r + hs;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = 4 * g + q;
        const double y = cl_yval(a[r][q], i, j, myscal[q]);
        if (i < rows) Qtop[i * TS_W + j] = (j < w) ? y : 0.0;
        if (8 * r < TS_W && wv == 0) {
          const bool in = i < w && j < w;
          Rf[i][j] = in ? cl_rval(a[r][q], i, j, mybeta[q]) : 0.0;
          Yt[i][j] = (i < w && j < w) ? y : 0.0;
        }
      }
    }
  }
  if (tid < TS_W) sg[tid] = 0.0;  // signs beyond w stay zero
  {
    constexpr int NL = TS_W * TS_W / TS_TREE_NT;
    double y[NL], t0[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + TS_TREE_NT * q, i = e & (TS_W - 1), j = e / TS_W;
      y[q] = (i < w && j < w)
                 ? ((i < j) ? 0.0 : ((i == j) ? 1.0 : V[ts_vrow(i, h1, vr2) + (long long)j * ldv]))
                 : 0.0;
      t0[q] = Tloc[e];  // zero beyond w (written so by the local factorisation)
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + TS_TREE_NT * q, i = e & (TS_W - 1), j = e / TS_W;
      Y0[i][j] = y[q];
      T0s[i][j] = t0[q];
    }
  }
  __syncthreads();
  // The 32 x 32 products below run over the zero-padded range, one 16 x 16
  // MFMA tile per wave on waves 0..3.
  const int wave = tid >> 6;
  const bool mw = wave < 4;
  const int ti = wave & 1, tj = wave >> 1, ri = tile_row(ti);
  if (mw) {  // Z = T_top Y_top(0:w, :)^T
    const d4 c = mfma_tile<TS_W>([&](int i, int k) { return Ts[i][k]; },
                                 [&](int k, int j) { return Yt[j][k]; }, ti, tj);
#pragma unroll
    for (int v = 0; v < 4; ++v) Z[ri][tile_col(tj, v)] = c[v];
  }
  __syncthreads();
  if (mw) {  // Q_top,0 = I - Y_top(0:32, :) Z (zero beyond w); Z to global memory
    const d4 c = mfma_tile<TS_W>([&](int i, int k) { return Yt[i][k]; },
                                 [&](int k, int j) { return Z[k][j]; }, ti, tj);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = tile_col(tj, v);
      Q0[ri][j] = (ri < w && j < w) ? ((ri == j ? 1.0 : 0.0) - c[v]) : 0.0;
      Zo[ri + TS_W * j] = Z[ri][j];
    }
  }
  __syncthreads();
  // Q_00 = Q_top,0 - Y_0 T_0 (Y_0^T Q_top,0): X2 = Y_0^T Q_top,0, X3 = T_0 X2
  double (*X2)[TS_W1] = Yt;
  double (*X3)[TS_W1] = Z;
  if (mw) {
    const d4 c = mfma_tile<TS_W>([&](int i, int k) { return Y0[k][i]; },
                                 [&](int k, int j) { return Q0[k][j]; }, ti, tj);
#pragma unroll
    for (int v = 0; v < 4; ++v) X2[ri][tile_col(tj, v)] = c[v];
  }
  __syncthreads();
  if (mw) {
    const d4 c = mfma_tile<TS_W>([&](int i, int k) { return T0s[i][k]; },
                                 [&](int k, int j) { return X2[k][j]; }, ti, tj);
#pragma unroll
    for (int v = 0; v < 4; ++v) X3[ri][tile_col(tj, v)] = c[v];
  }
  __syncthreads();
  if (mw) {
    const d4 c = mfma_tile<TS_W>([&](int i, int k) { return Y0[i][k]; },
                                 [&](int k, int j) { return X3[k][j]; }, ti, tj);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = tile_col(tj, v);
      X2[ri][j] = Q0[ri][j] - c[v];  // Q_00 (zero beyond w)
    }
  }
  __syncthreads();
  // LU of Q_00 - S in LDS by all threads, one barrier per step: the sign s_k
  // is chosen so that |pivot| >= 1, and the trailing block is updated with
  // the unscaled column k (L(i, k) = X2(i, k) / pivot_k afterwards).
  for (int k = 0; k < w; ++k) {
    const double akk = X2[k][k];
    const double sk = (akk >= 0.0) ? -1.0 : 1.0;
    const double piv = akk - sk;
    const double rp = 1.0 / piv;
    if (tid == 0) { sg[k] = sk; pv[k] = piv; }
#pragma unroll
    for (int q = 0; q < TS_W * TS_W / TS_TREE_NT; ++q) {
      const int e = tid + TS_TREE_NT * q;
      const int i = e & (TS_W - 1), jj = e / TS_W;
      if (i > k && jj > k && i < w && jj < w) X2[i][jj] = fma(-X2[i][k] * rp, X2[k][jj], X2[i][jj]);
    }
    __syncthreads();
  }
  // U (pivots on the diagonal) and L^T (unit diagonal), identity beyond w, for
  // the inverses; L to global memory
  double (*Us)[TS_W1] = T0s;  // U
  double (*Lt)[TS_W1] = Y0;   // L^T
  double (*Ui)[TS_W1] = Q0;   // U^{-1}
  double (*Li)[TS_W1] = Z;    // L1^{-T}
  for (int e = tid; e < TS_W * TS_W; e += TS_TREE_NT) {
    const int i = e & (TS_W - 1), j = e / TS_W;
    const bool in = i < w && j < w;
    Us[i][j] = in ? ((i < j) ? X2[i][j] : ((i == j) ? pv[i] : 0.0)) : ((i == j) ? 1.0 : 0.0);
    Lt[i][j] = in ? ((i < j) ? X2[j][i] / pv[i] : ((i == j) ? 1.0 : 0.0)) : ((i == j) ? 1.0 : 0.0);
    Lo[i + TS_W * j] = in ? ((i > j) ? X2[i][j] / pv[j] : ((i == j) ? 1.0 : 0.0)) : 0.0;
  }
  __syncthreads();
  lds_upper_inverse32x2(Us, Ui, Lt, Li, Ts);
  if (mw) {  // T = -U S L1^{-T} (upper)
    const d4 c = mfma_tile<TS_W>([&](int i, int k) { return Us[i][k] * sg[k]; },
                                 [&](int k, int j) { return Li[k][j]; }, ti, tj);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = tile_col(tj, v);
      Tfin[ri + (long long)j * TS_W] = (ri <= j && ri < w && j < w) ? -c[v] : 0.0;
    }
  }
  // R = S R_tsqr into the matrix (top w logical rows = segment 1), zeros below the diagonal
  for (int e = tid; e < w * w; e += TS_TREE_NT) {
    const int i = e % w, j = e / w;
    M[ts_phys(i, h1, r1a, r2a) + (long long)(c0 + j) * ldm] = (i <= j) ? sg[i] * Rf[i][j] : 0.0;
  }
  // U^{-1} (zero beyond w) and S for the row expansion (L1 was written above)
  for (int e = tid; e < TS_W * TS_W; e += TS_TREE_NT) {
    const int i = e % TS_W, j = e / TS_W;
    Uo[e] = (i < w && j < w) ? Ui[i][j] : 0.0;
  }
  if (tid < w) So[tid] = sg[tid];
}

// C: rows of Q and of V = Q U^{-1}; zero the annihilated panel entries.
// With M2 = T_p Y_p(0:w, :)^T Q_top,p, the row i of the panel's Q is
// q = [Q_top,p; 0](i, :) - y M2 (y = Y_p(i, :)), so v = q U^{-1} =
// Q3(i, :) - y M3 with Q3 = Q_top,p U^{-1} and M3 = M2 U^{-1} formed once per
// block (32 x 32 products, one MFMA tile per wave); the block's rows of V are
// then one 256 x 32 x 32 product, Y_p read straight from V in MFMA fragments.
__global__ __launch_bounds__(TS_NT) void tsqr_expand_kernel(
    double* M, long long ldm, long long sM, int c0, int w, int h1, int r1a, int r2a, int h, int P,
    double* V, long long ldv, long long sV, int vr2, const double* Tloc, const double* Ytop,
    const double* Zg, const double* Uinv, const double* Lo, long long sScr) {
  __shared__ double Qt[TS_W][TS_W1];
  __shared__ double Us[TS_W][TS_W1];  // U^{-1}
  __shared__ double M1[TS_W][TS_W1];  // Y_top,p, then Y_p^T Q_top,p, then M3
  __shared__ double M2[TS_W][TS_W1];  // Z, then M2
  __shared__ double Q3[TS_W][TS_W1];
  __shared__ double Yp[TS_W][TS_W1];  // Y_p(0:32, :)
  __shared__ double Tp[TS_W][TS_W1];  // T_p
  const int p = blockIdx.x;
  const long long b = blockIdx.y;
  M += b * sM;
  V += b * sV;
  Tloc += b * sScr;
  Ytop += b * sScr;
  Zg += b * sScr;
  Uinv += b * sScr;
  Lo += b * sScr;
  const int tid = threadIdx.x;
  const int i0 = p * TS_MB;
  const int rows = min(TS_MB, h - i0);
  const int wy = min(w, rows);  // rows of Y_p that meet [Q_top,p; 0]
  const double* Tpg = Tloc + (long long)p * TS_W * TS_W;
  {
    // all loads of a thread in flight at once, then the LDS stores
    constexpr int NL = TS_W * TS_W / TS_NT;
    double l1[NL], l2[NL], l3[NL], l4[NL], l5[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + TS_NT * q, i = e % TS_W, j = e / TS_W;
      const bool in = i < w && j < w;
      l1[q] = in ? Ytop[(p * w + i) * TS_W + j] : 0.0;
      l2[q] = Zg[e];
      l3[q] = in ? Uinv[e] : 0.0;
      l4[q] = (i < wy && j < w)
                  ? ((i > j) ? V[ts_vrow(i0 + i, h1, vr2) + (long long)j * ldv] : ((i == j) ? 1.0 : 0.0))
                  : 0.0;
      l5[q] = (in && i <= j) ? Tpg[e] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + TS_NT * q, i = e % TS_W, j = e / TS_W;
      M1[i][j] = l1[q];
      M2[i][j] = l2[q];
      Us[i][j] = l3[q];
      Yp[i][j] = l4[q];
      Tp[i][j] = l5[q];
    }
  }
  __syncthreads();
  const int wave = tid >> 6;
  const int ti = wave & 1, tj = wave >> 1, ri = tile_row(ti);
  {  // Q_top,p = [I; 0]_p - Y_top,p Z
    const d4 c = mfma_tile<TS_W>([&](int i, int k) { return M1[i][k]; },
                                 [&](int k, int j) { return M2[k][j]; }, ti, tj);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = tile_col(tj, v);
      Qt[ri][j] = (ri < w && j < w) ? (((p == 0 && ri == j) ? 1.0 : 0.0) - c[v]) : 0.0;
    }
  }
  __syncthreads();
  {  // M1 = Y_p(0:32, :)^T Q_top,p and Q3 = Q_top,p U^{-1}
    const d4 c = mfma_tile<TS_W>([&](int i, int k) { return Yp[k][i]; },
                                 [&](int k, int j) { return Qt[k][j]; }, ti, tj);
    const d4 c3 = mfma_tile<TS_W>([&](int i, int k) { return Qt[i][k]; },
                                  [&](int k, int j) { return Us[k][j]; }, ti, tj);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = tile_col(tj, v);
      M1[ri][j] = c[v];
      Q3[ri][j] = c3[v];
    }
  }
  __syncthreads();
  {  // M2 = T_p M1
    const d4 c = mfma_tile<TS_W>([&](int i, int k) { return Tp[i][k]; },
                                 [&](int k, int j) { return M1[k][j]; }, ti, tj);
#pragma unroll
    for (int v = 0; v < 4; ++v) M2[ri][tile_col(tj, v)] = c[v];
  }
  __syncthreads();
  double (*M3)[TS_W1] = M1;
  {  // M3 = M2 U^{-1}
    const d4 c = mfma_tile<TS_W>([&](int i, int k) { return M2[i][k]; },
                                 [&](int k, int j) { return Us[k][j]; }, ti, tj);
#pragma unroll
    for (int v = 0; v < 4; ++v) M3[ri][tile_col(tj, v)] = c[v];
  }
  __syncthreads();
  // rows of V: V(i, :) = Q3(i, :) - Y_p(i, :) M3 (Q3 is zero beyond row 31); on
  // block 0 the first w rows are L1.  Each wave owns row tiles wave, wave + 4, ...
  // and both column tiles, and reads its Y fragments from V before it writes V.
  const int lane = tid & 63;
  const int lr = lane & 15, lk = lane >> 4;
  // the local Y rows of every row tile this wave rewrites, loaded before any
  // of them is overwritten (each tile rewrites only its own rows)
  constexpr int NRT = TS_MB / 64, NK = TS_W / 4;
  double yv[NRT][NK];
#pragma unroll
  for (int it = 0; it < NRT; ++it) {
    const int il = 16 * (wave + 4 * it) + lr;
    const bool rin = il < rows;
    const long long vi = rin ? ts_vrow(i0 + il, h1, vr2) : 0;
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      const int k = 4 * s + lk;
      yv[it][s] = (rin && k < w) ? V[vi + (long long)k * ldv] : 0.0;
    }
  }
#pragma unroll
  for (int it = 0; it < NRT; ++it) {
    const int rt = wave + 4 * it;
    if (rt * 16 >= rows) break;
    const int il = 16 * rt + lr;  // the row this lane feeds
    const bool rin = il < rows;
    const long long vi = rin ? ts_vrow(i0 + il, h1, vr2) : 0;
    d4 c0t = {0.0, 0.0, 0.0, 0.0}, c1t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      const int k = 4 * s + lk;
      c0t = __builtin_amdgcn_mfma_f64_16x16x4f64(M3[k][lr], yv[it][s], c0t, 0, 0, 0);
      c1t = __builtin_amdgcn_mfma_f64_16x16x4f64(M3[k][16 + lr], yv[it][s], c1t, 0, 0, 0);
    }
    // lane l item v holds row 16 rt + l % 16, column 16 tj + 4 v + l / 16
    if (rin) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int j = 16 * t + 4 * v + lk;
          if (j < w) {
            double val;
            if (p == 0 && il < w) val = Lo[il + TS_W * j];
            else val = ((il < TS_W) ? Q3[il][j] : 0.0) - (t ? c1t[v] : c0t[v]);
            V[vi + (long long)j * ldv] = val;
          }
        }
      }
    }
  }
  if (tid < rows) {
    const int gi = i0 + tid;
    if (gi >= w) {
      const long long pr = ts_phys(gi, h1, r1a, r2a);
      for (int j = 0; j < w; ++j) M[pr + (long long)(c0 + j) * ldm] = 0.0;
    }
  }
}

bool tsqr_panel_fits(int h, int w) { return w <= TS_W && w >= 1 && h >= w && h <= TS_PMAX * TS_MB; }

void tsqr_panel(int batch, double* M, long long ldm, long long sM, int c0, int w, int r1a, int r1b,
                int r2a, int r2b, double* V, long long ldv, long long sV, int vr2, double* T,
                long long sT, const TsqrScratch& sc, hipStream_t s) {
  const int h1 = r1b - r1a, h2 = r2b - r2a, h = h1 + h2;
  if (vr2 < 0) vr2 = h1;
  if (!tsqr_panel_fits(h, w)) throw ArgError("tsqr_panel: panel too tall");
  const int P = (h + TS_MB - 1) / TS_MB;
  const double ww = (double)w * w;
  {
    ProfScope prof("tsqr_local", s, batch * (2.0 * h * ww - P * 2.0 * ww * w / 3.0),
                   batch * 8.0 * 2.0 * h * w);
    if (h <= 2 * TS_MB && P > 1) {
      // up to 512 rows: one block on eight waves, finished directly
      hipLaunchKernelGGL(tsqr_local_kernel<8>, dim3(1, batch), dim3(512), 0, s, M, ldm, sM, c0, w,
                         h1, r1a, r2a, h, 1, V, ldv, sV, vr2, sc.Tloc, sc.Rstack, sc.stride, 1, T,
                         sT);
      ZCSD_CHECK_LAUNCH();
      return;
    }
    hipLaunchKernelGGL(tsqr_local_kernel<TS_NT / 64>, dim3(P, batch), dim3(TS_NT), 0, s, M, ldm, sM,
                       c0, w, h1, r1a, r2a, h, P, V, ldv, sV, vr2, sc.Tloc, sc.Rstack, sc.stride,
                       P == 1 ? 1 : 0, T, sT);
    ZCSD_CHECK_LAUNCH();
  }
  if (P == 1) return;  // one block: its Householder QR is the panel's
  {
    ProfScope prof("tsqr_tree", s, batch * (4.0 * P * ww * w + 4.0 * ww * w),
                   batch * 8.0 * 2.0 * P * ww);
    // row slots per lane: the 8 waves hold 64 RQ rows >= the P w stacked rows,
    // and wave 0 holds the first 32 (RQ >= 4)
#define ZCSD_TREE_LAUNCH(RQ_)                                                                    \
  hipLaunchKernelGGL(tsqr_tree_kernel<RQ_>, dim3(batch), dim3(TS_TREE_NT), 0, s, M, ldm, sM, c0, w, \
                     h1, r1a, r2a, P, V, ldv, sV, vr2, sc.Tloc, sc.Rstack, sc.Qtop, sc.Z, sc.U,    \
                     sc.L, sc.S, sc.stride, T, sT)
    if (P <= 8) ZCSD_TREE_LAUNCH(4);
    else if (P <= 12) ZCSD_TREE_LAUNCH(6);
    else ZCSD_TREE_LAUNCH(TS_TREE_RQ);
#undef ZCSD_TREE_LAUNCH
    ZCSD_CHECK_LAUNCH();
  }
  {
    ProfScope prof("tsqr_expand", s, batch * 3.0 * h * ww, batch * 8.0 * 3.0 * h * w);
    hipLaunchKernelGGL(tsqr_expand_kernel, dim3(P, batch), dim3(TS_NT), 0, s, M, ldm, sM, c0, w, h1,
                       r1a, r2a, h, P, V, ldv, sV, vr2, sc.Tloc, sc.Qtop, sc.Z, sc.U, sc.L,
                       sc.stride);
    ZCSD_CHECK_LAUNCH();
  }
}

size_t tsqr_scratch_bytes(int batch) {
  const long long per_R = (long long)TS_PMAX * TS_W * TS_W;
  const long long stride = 4 * per_R + 3 * TS_W * TS_W + TS_W;
  return (((size_t)batch * stride * sizeof(double) + 255) / 256) * 256;
}

TsqrScratch tsqr_scratch_alloc(Arena& ar, int batch) {
  TsqrScratch sc;
  const long long per_R = (long long)TS_PMAX * TS_W * TS_W;  // Rstack, Qtop: (P w) x w
  sc.stride = 4 * per_R + 3 * TS_W * TS_W + TS_W;
  double* base = ar.dalloc((size_t)batch * sc.stride);
  sc.Rstack = base;
  sc.Qtop = base + per_R;
  sc.Tloc = base + 2 * per_R;  // P blocks of w x w
  sc.Z = base + 3 * per_R;     // 32 x 32
  sc.U = base + 4 * per_R;
  sc.L = sc.U + TS_W * TS_W;
  sc.S = sc.L + TS_W * TS_W;
  return sc;
}

}  // namespace zcsd
