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
// Each stage is parallel over rows; only the w x w pieces are sequential.
// The Householder factorisations keep the matrix in registers, one row (or a
// few) per thread: a step needs the dot products of the pivot column with all
// 32 columns, which one butterfly over the wave and a 4-way sum across the
// waves deliver together, so a step costs two barriers.
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
constexpr int TS_TREE_RPT = (TS_PMAX * TS_W + TS_NT - 1) / TS_NT;  // rows per thread in the tree

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

// One DPP halving step: partner lanes exchange the halves they do not keep;
// `hi` lanes keep the upper half.  The halves are chosen with a bit mask, not
// with a conditional on the array index (which the compiler may turn into a
// dynamic index and demote x to memory).
template <int CTRL, int HS>
__device__ __forceinline__ void dpp_halve(double (&x)[TS_W], bool hi) {
  const long long m = hi ? -1LL : 0LL;
#pragma unroll
  for (int k = 0; k < HS; ++k) {
    const long long lo = __double_as_longlong(x[k]), up = __double_as_longlong(x[k + HS]);
    const double keep = __longlong_as_double((up & m) | (lo & ~m));
    const double send = __longlong_as_double((lo & m) | (up & ~m));
    x[k] = keep + dpp_f64<CTRL>(send);
  }
}

// Sum over the 64 lanes of a wave of 32 values per lane by recursive halving:
// partners lane ^ 32 and lane ^ 16 (permlane swaps), lane ^ 8 (DPP row_ror:8),
// lane ^ 7 within 8-lane groups (row_half_mirror), lane ^ 2 and a last pairwise
// add with lane ^ 1 (quad_perm).  The partner of every step agrees with the lane
// on all bits used before, so lane l returns the sum of x[(l >> 1) & 31].
__device__ __forceinline__ double wave_sum32(double (&x)[TS_W]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < 16; ++k) x[k] = swap_sum<true>(x[k], x[k + 16]);
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = swap_sum<false>(x[k], x[k + 8]);
  dpp_halve<0x128, 4>(x, (lane & 8) != 0);  // row_ror:8
  dpp_halve<0x141, 2>(x, (lane & 4) != 0);  // row_half_mirror
  dpp_halve<0x4E, 1>(x, (lane & 2) != 0);   // quad_perm [2,3,0,1]
  return x[0] + dpp_f64<0xB1>(x[0]);        // quad_perm [1,0,3,2]
}

// Householder QR of a rows x w matrix (w <= 32) held in registers: row
// i = threadIdx.x + TS_NT * r is a[r][:]; entries beyond rows / w are zero.
// Step t forms d_j = sum_{i >= t} a_it a_ij for every j at once; with
// alpha = a_tt, beta = -sign(alpha) sqrt(d_t), v = (a_t - beta e_t)/(alpha - beta)
// (v_t = 1), tau = (beta - alpha)/beta, the products v^T a_j = (d_j - beta a_tj)
// / (alpha - beta) serve both the update a_j -= tau v (v^T a_j) (j > t) and the
// column t of T, T(0:t, t) = -tau T(0:t, 0:t) Y(:, 0:t)^T v (k < t).
// On return the rows hold R (upper, diagonal beta) and the vectors below the
// diagonal (unit diagonal implicit), and T is in Ts.
// One barrier per step: the per-wave partial sums and the pivot row go to
// double-buffered LDS (a buffer is rewritten two steps later, after every wave
// has passed the next barrier), each lane reads back the sums of its own
// column, and the pivot scalars and the update coefficients are broadcast with
// readlane.  LDS: red[2 * 4 * 32], rowb[2 * 32], zb[32].
template <int t, int RPT>
__device__ __forceinline__ void reg_householder_step(double (&a)[RPT][TS_W], int rows,
                                                     double (*Ts)[TS_W1], double* red, double* rowb,
                                                     double* zb) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int buf = t & 1;
  double* rb = red + buf * 4 * TS_W;     // [wave][j] partial sums of this step
  double* pr = rowb + buf * TS_W;        // pivot row a(t, :)
  double x[TS_W];
#pragma unroll
  for (int j = 0; j < TS_W; ++j) x[j] = 0.0;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + TS_NT * r;
    if (i >= t && i < rows) {
      const double ait = a[r][t];
#pragma unroll
      for (int j = 0; j < TS_W; ++j) x[j] = fma(ait, a[r][j], x[j]);
    }
    if (i == t) {
#pragma unroll
      for (int j = 0; j < TS_W; ++j) pr[j] = a[r][j];
    }
  }
  const double sj = wave_sum32(x);
  const int jl = (lane >> 1) & 31;  // the column this lane's sum belongs to
  if ((lane & 1) == 0) rb[wave * TS_W + jl] = sj;
  __syncthreads();
  // d_j and a(t, j) for this lane's column; the pivot's through readlane
  const double dj = (rb[jl] + rb[TS_W + jl]) + (rb[2 * TS_W + jl] + rb[3 * TS_W + jl]);
  const double atj = pr[jl];
  const double dt = readlane_f64(dj, 2 * t), alpha = readlane_f64(atj, 2 * t);
  double tau = 0.0, beta = 0.0, scal = 0.0;
  if (dt > 0.0) {
    const double nrm = sqrt(dt);
    beta = alpha >= 0.0 ? -nrm : nrm;
    tau = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
  // v^T a_j (j > t: the update) and y_j^T v (j < t: the T column), this lane's j
  const double wl = scal * (dj - beta * atj);
  double tv[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + TS_NT * r;
    const double v = (i > t && i < rows) ? scal * a[r][t] : ((i == t) ? 1.0 : 0.0);
    tv[r] = tau * v;
    if (i > t && i < rows) a[r][t] = v;
    else if (i == t) a[r][t] = beta;
  }
#pragma unroll
  for (int j = t + 1; j < TS_W; ++j) {
    const double wj = readlane_f64(wl, 2 * j);
#pragma unroll
    for (int r = 0; r < RPT; ++r) a[r][j] = fma(-tv[r], wj, a[r][j]);
  }
  // column t of T, by wave 0 (its even lanes hold every y_k^T v)
  if (wave == 0) {
    if ((lane & 1) == 0) zb[jl] = wl;
    __builtin_amdgcn_wave_barrier();
    if (lane < t) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < t; ++k) s = fma(Ts[lane][k], zb[k], s);
      Ts[lane][t] = -tau * s;
    } else if (lane == t) {
      Ts[t][t] = tau;
    }
  }
}

// the 32 steps, unrolled at compile time so that every register index is static
template <int t, int RPT>
__device__ __forceinline__ void reg_householder_steps(double (&a)[RPT][TS_W], int rows, int w,
                                                      double (*Ts)[TS_W1], double* red,
                                                      double* rowb, double* zb) {
  if constexpr (t < TS_W) {
    if (t < w) {
      reg_householder_step<t, RPT>(a, rows, Ts, red, rowb, zb);
      reg_householder_steps<t + 1, RPT>(a, rows, w, Ts, red, rowb, zb);
    }
  }
}

// Ts (LDS, 32 x 33) receives T; it is zeroed here and complete after the
// caller's next barrier.
template <int RPT>
__device__ void reg_householder(double (&a)[RPT][TS_W], int rows, int w, double (*Ts)[TS_W1],
                                double* red, double* rowb, double* zb) {
  for (int e = threadIdx.x; e < TS_W * TS_W1; e += TS_NT) (&Ts[0][0])[e] = 0.0;
  __syncthreads();
  reg_householder_steps<0, RPT>(a, rows, w, Ts, red, rowb, zb);
}
// ---------------------------------------------------------------------------
// A: local QR of every row block
__global__ __launch_bounds__(TS_NT) void tsqr_local_kernel(
    const double* M, long long ldm, long long sM, int c0, int w, int h1, int r1a, int r2a, int h,
    int P, double* V, long long ldv, long long sV, int vr2, double* Tloc, double* Rstack,
    long long sScr) {
  __shared__ double red[2 * 4 * TS_W], rowb[2 * TS_W], zb[TS_W];
  __shared__ double Ts[TS_W][TS_W1];
  const int p = blockIdx.x;
  const long long b = blockIdx.y;
  M += b * sM;
  V += b * sV;
  const int i0 = p * TS_MB;
  const int rows = min(TS_MB, h - i0);
  const int tid = threadIdx.x;
  double a[1][TS_W];
  {
    const long long pr = (tid < rows) ? ts_phys(i0 + tid, h1, r1a, r2a) : 0;
#pragma unroll
    for (int j = 0; j < TS_W; ++j)
      a[0][j] = (tid < rows && j < w) ? M[pr + (long long)(c0 + j) * ldm] : 0.0;
  }
  reg_householder<1>(a, rows, w, Ts, red, rowb, zb);
  // Y_p (unit lower trapezoidal) into V's rows, R_p (upper w x w, zero rows
  // beyond the block), T_p
  if (tid < rows) {
#pragma unroll
    for (int j = 0; j < TS_W; ++j)
      if (j < w)
        V[ts_vrow(i0 + tid, h1, vr2) + (long long)j * ldv] = (tid < j) ? 0.0 : ((tid == j) ? 1.0 : a[0][j]);
  }
  const int ldr = P * TS_W;
  if (tid < w) {
    double* Rp = Rstack + b * sScr;
#pragma unroll
    for (int j = 0; j < TS_W; ++j)
      if (j < w) Rp[(p * w + tid) + (long long)j * ldr] = (j >= tid && tid < rows) ? a[0][j] : 0.0;
  }
  __syncthreads();
  double* Tp = Tloc + b * sScr + (long long)p * TS_W * TS_W;
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) Tp[e] = Ts[e % TS_W][e / TS_W];
}

// B: QR of the stacked R factors (registers), explicit Q_top, reconstruction
// pieces (w x w work in LDS).
__global__ __launch_bounds__(TS_NT) void tsqr_tree_kernel(
    double* M, long long ldm, long long sM, int c0, int w, int h1, int r1a, int r2a, int P,
    const double* V, long long ldv, long long sV, int vr2, const double* Tloc, const double* Rstack,
    double* Qtop, double* Zo, double* Uo, double* Lo, double* So, long long sScr, double* Tfin,
    long long sT) {
  __shared__ double red[2 * 4 * TS_W], rowb[2 * TS_W], zb[TS_W];
  __shared__ double Ts[TS_W][TS_W1];  // T_top
  __shared__ double Yt[TS_W][TS_W1];  // Y_top(0:w, 0:w), then X2
  __shared__ double Z[TS_W][TS_W1];   // T_top Y_top(0:w, :)^T, then L1^{-T}
  __shared__ double Rf[TS_W][TS_W1];  // R_tsqr
  __shared__ double Q0[TS_W][TS_W1];  // Q_top,0, then Q_00 and its LU
  __shared__ double Y0[TS_W][TS_W1];  // Y_0(0:w, 0:w) of block 0
  __shared__ double T0s[TS_W][TS_W1]; // T_0 of block 0, then U
  __shared__ double sg[TS_W];
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
  const int ldr = P * TS_W;
  double a[TS_TREE_RPT][TS_W];
#pragma unroll
  for (int r = 0; r < TS_TREE_RPT; ++r) {
    const int i = tid + TS_NT * r;
#pragma unroll
    for (int j = 0; j < TS_W; ++j) a[r][j] = (i < rows && j < w) ? Rstack[i + (long long)j * ldr] : 0.0;
  }
  reg_householder<TS_TREE_RPT>(a, rows, w, Ts, red, rowb, zb);
  // R_tsqr and Y_top(0:w, 0:w) from the first w rows (rows w..31 belong to the
  // next block: zero here), Y_0(0:w, 0:w) and T_0 of block 0
  if (tid < TS_W) {
    const bool in = tid < w;
#pragma unroll
    for (int j = 0; j < TS_W; ++j) {
      Rf[tid][j] = (in && j >= tid) ? a[0][j] : 0.0;
      Yt[tid][j] = in ? ((j < tid) ? a[0][j] : ((j == tid) ? 1.0 : 0.0)) : 0.0;
    }
  }
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e & (TS_W - 1), j = e / TS_W;
    Y0[i][j] = (i < w && j < w)
                   ? ((i < j) ? 0.0 : ((i == j) ? 1.0 : V[ts_vrow(i, h1, vr2) + (long long)j * ldv]))
                   : 0.0;
    T0s[i][j] = Tloc[e];  // zero beyond w (written so by the local factorisation)
    Q0[i][j] = 0.0;
  }
  __syncthreads();
  // Z = T_top Y_top(0:w, :)^T; all 32 x 32 products below run over the full
  // zero-padded range so that the loops unroll
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e & (TS_W - 1), j = e / TS_W;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < TS_W; ++q) s = fma(Ts[i][q], Yt[j][q], s);
    Z[i][j] = s;
  }
  __syncthreads();
  // Y_top (unit lower trapezoidal, explicit) and Z to global memory: every
  // expansion block forms its own rows of Q_top = [I; 0] - Y_top Z.  Here only
  // Q_top,0 (rows 0..31) is formed, for Q_00.
#pragma unroll
  for (int r = 0; r < TS_TREE_RPT; ++r) {
    const int i = tid + TS_NT * r;
    if (i < rows) {
#pragma unroll
      for (int k = 0; k < TS_W; ++k)
        if (k < w) Qtop[i + (long long)k * ldr] = (i > k) ? a[r][k] : ((i == k) ? 1.0 : 0.0);
    }
  }
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e & (TS_W - 1), j = e / TS_W;
    Zo[e] = Z[i][j];
    double q = (i == j) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < TS_W; ++k) q = fma(-Yt[i][k], Z[k][j], q);
    Q0[i][j] = (i < w && j < w) ? q : 0.0;
  }
  __syncthreads();
  // Q_00 = Q_top,0 - Y_0 T_0 (Y_0^T Q_top,0): X2 = Y_0^T Q_top,0, X3 = T_0 X2
  double (*X2)[TS_W1] = Yt;
  double (*X3)[TS_W1] = Z;
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e & (TS_W - 1), j = e / TS_W;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < TS_W; ++q) s = fma(Y0[q][i], Q0[q][j], s);
    X2[i][j] = s;
  }
  __syncthreads();
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e & (TS_W - 1), j = e / TS_W;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < TS_W; ++q) s = fma(T0s[i][q], X2[q][j], s);
    X3[i][j] = s;
  }
  __syncthreads();
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e & (TS_W - 1), j = e / TS_W;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < TS_W; ++q) s = fma(Y0[i][q], X3[q][j], s);
    X2[i][j] = Q0[i][j] - s;  // Q_00 (zero beyond w)
  }
  __syncthreads();
  // Wave 0, lane i < w holding row i in registers: LU of Q_00 - S with the
  // pivot sign chosen so that |pivot| >= 1, then L1^{-1} and U^{-1} column by
  // column (lane j owns column j); pivot rows are broadcast with readlane.
  double (*Li)[TS_W1] = Z;   // L1^{-T}
  double (*Ui)[TS_W1] = Q0;  // U^{-1}
  double (*Us)[TS_W1] = T0s; // U
  if (tid < 64) {
    const int lane = tid;
    const bool own = lane < w;
    double row[TS_W];
#pragma unroll
    for (int j = 0; j < TS_W; ++j) row[j] = own ? X2[lane][j] : 0.0;
    if (lane < TS_W) sg[lane] = 0.0;  // signs beyond w stay zero
#pragma unroll
    for (int k = 0; k < TS_W; ++k) {
      if (k < w) {
        const double akk = readlane_f64(row[k], k);
        const double sk = (akk >= 0.0) ? -1.0 : 1.0;
        const double piv = akk - sk;
        const double rp = 1.0 / piv;
        if (lane == 0) sg[k] = sk;
        if (lane == k) row[k] = piv;
        double pr[TS_W];
#pragma unroll
        for (int j = k + 1; j < TS_W; ++j) pr[j] = readlane_f64(row[j], k);
        if (lane > k && own) {
          const double l = row[k] * rp;
          row[k] = l;
#pragma unroll
          for (int j = k + 1; j < TS_W; ++j) row[j] = fma(-l, pr[j], row[j]);
        }
      }
    }
    // row now holds L (strictly below the diagonal, unit diagonal implicit) and U
    double xc[TS_W];
    // L1^{-1}: x_i = e_i - sum_{k < i} L_ik x_k (column `lane`)
#pragma unroll
    for (int i = 0; i < TS_W; ++i) {
      double x = (lane == i) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) x = fma(-readlane_f64(row[k], i), xc[k], x);
      xc[i] = (i < w) ? x : 0.0;
    }
    if (lane < TS_W) {
#pragma unroll
      for (int i = 0; i < TS_W; ++i) Li[lane][i] = own ? xc[i] : 0.0;  // L1^{-T}(lane, i) = L1^{-1}(i, lane)
    }
    // U^{-1}: x_i = (e_i - sum_{k > i} U_ik x_k) / U_ii (column `lane`)
#pragma unroll
    for (int i = TS_W - 1; i >= 0; --i) {
      double x = 0.0;
      if (i < w) {
        x = (lane == i) ? 1.0 : 0.0;
#pragma unroll
        for (int k = i + 1; k < TS_W; ++k) x = fma(-readlane_f64(row[k], i), xc[k], x);
        x *= 1.0 / readlane_f64(row[i], i);
      }
      xc[i] = x;
    }
    if (lane < TS_W) {
#pragma unroll
      for (int i = 0; i < TS_W; ++i) {
        Ui[i][lane] = own ? xc[i] : 0.0;
        Us[lane][i] = (own && i >= lane) ? row[i] : 0.0;
        Lo[lane + i * TS_W] = own ? ((i < lane) ? row[i] : ((i == lane) ? 1.0 : 0.0)) : 0.0;
      }
    }
  }
  __syncthreads();
  // T = -U S L1^{-T} (upper)
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e & (TS_W - 1), j = e / TS_W;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < TS_W; ++q) s = fma(Us[i][q] * sg[q], Li[q][j], s);
    Tfin[i + (long long)j * TS_W] = (i <= j) ? -s : 0.0;
  }
  // R = S R_tsqr into the matrix (top w logical rows = segment 1), zeros below the diagonal
  for (int e = tid; e < w * w; e += TS_NT) {
    const int i = e % w, j = e / w;
    M[ts_phys(i, h1, r1a, r2a) + (long long)(c0 + j) * ldm] = (i <= j) ? sg[i] * Rf[i][j] : 0.0;
  }
  // U^{-1} and S for the row expansion (L1 was written above)
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) Uo[e] = Ui[e % TS_W][e / TS_W];
  if (tid < w) So[tid] = sg[tid];
}

// C: rows of Q and of V = Q U^{-1}; zero the annihilated panel entries.
// With M2 = T_p Y_p(0:w, :)^T Q_top,p, the row i of the panel's Q is
// q = [Q_top,p; 0](i, :) - y M2 (y = Y_p(i, :)), so v = q U^{-1} =
// Q3(i, :) - y M3 with Q3 = Q_top,p U^{-1} and M3 = M2 U^{-1} formed once per
// block; y stays in registers and v is produced one column at a time.
__global__ __launch_bounds__(TS_NT) void tsqr_expand_kernel(
    double* M, long long ldm, long long sM, int c0, int w, int h1, int r1a, int r2a, int h, int P,
    double* V, long long ldv, long long sV, int vr2, const double* Tloc, const double* Ytop,
    const double* Zg, const double* Uinv, const double* Lo, long long sScr) {
  __shared__ double Qt[TS_W][TS_W1];
  __shared__ double Us[TS_W][TS_W1];  // U^{-1}
  __shared__ double M1[TS_W][TS_W1];  // Y_p^T Q_top,p, then M3
  __shared__ double M2[TS_W][TS_W1];
  __shared__ double Q3[TS_W][TS_W1];
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
  const int ldr = P * TS_W;
  const double* Tp = Tloc + (long long)p * TS_W * TS_W;
  // Q_top,p = [I; 0]_p - Y_top,p Z (Y_top,p = rows p w .. p w + w - 1 of Y_top);
  // M1 and M2 hold Y_top,p and Z until Qt is formed
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e % TS_W, j = e / TS_W;
    const bool in = i < w && j < w;
    M1[i][j] = in ? Ytop[(p * w + i) + (long long)j * ldr] : 0.0;
    M2[i][j] = Zg[e];
    Us[i][j] = in ? Uinv[i + j * TS_W] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e % TS_W, j = e / TS_W;
    double q = (p == 0 && i == j) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < TS_W; ++k) q = fma(-M1[i][k], M2[k][j], q);
    Qt[i][j] = (i < w && j < w) ? q : 0.0;
  }
  __syncthreads();
  // M1 = Y_p(0:wy, :)^T Q_top,p(0:wy, :) (Y_p unit lower on its first rows);
  // Q3 = Q_top,p U^{-1}
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e % TS_W, j = e / TS_W;
    double s = 0.0, s3 = 0.0;
    if (i < w && j < w) {
      for (int q = i; q < wy; ++q)
        s = fma((q == i) ? 1.0 : V[ts_vrow(i0 + q, h1, vr2) + (long long)i * ldv], Qt[q][j], s);
      for (int q = 0; q <= j; ++q) s3 = fma(Qt[i][q], Us[q][j], s3);
    }
    M1[i][j] = s;
    Q3[i][j] = s3;
  }
  __syncthreads();
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e % TS_W, j = e / TS_W;
    double s = 0.0;  // rows/columns beyond w stay exactly zero
    if (i < w && j < w)
      for (int q = i; q < w; ++q) s = fma(Tp[i + q * TS_W], M1[q][j], s);
    M2[i][j] = s;
  }
  __syncthreads();
  double (*M3)[TS_W1] = M1;
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e % TS_W, j = e / TS_W;
    double s = 0.0;
    if (i < w && j < w)
      for (int q = 0; q <= j; ++q) s = fma(M2[i][q], Us[q][j], s);
    M3[i][j] = s;
  }
  __syncthreads();
  if (tid < rows) {
    const int i = tid;
    const int gi = i0 + i;
    const long long vi = ts_vrow(gi, h1, vr2);
    if (p == 0 && i < w) {
      for (int j = 0; j < w; ++j) V[vi + (long long)j * ldv] = Lo[i + j * TS_W];
    } else {
      double y[TS_W];
#pragma unroll
      for (int k = 0; k < TS_W; ++k) y[k] = (k < w) ? V[vi + (long long)k * ldv] : 0.0;
#pragma unroll 2
      for (int j = 0; j < w; ++j) {
        double v = (i < TS_W) ? Q3[i][j] : 0.0;
#pragma unroll
        for (int k = 0; k < TS_W; ++k) v = fma(-y[k], M3[k][j], v);
        V[vi + (long long)j * ldv] = v;
      }
    }
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
    hipLaunchKernelGGL(tsqr_local_kernel, dim3(P, batch), dim3(TS_NT), 0, s, M, ldm, sM, c0, w, h1,
                       r1a, r2a, h, P, V, ldv, sV, vr2, sc.Tloc, sc.Rstack, sc.stride);
    ZCSD_CHECK_LAUNCH();
  }
  {
    ProfScope prof("tsqr_tree", s, batch * (4.0 * P * ww * w + 4.0 * ww * w),
                   batch * 8.0 * 2.0 * P * ww);
    hipLaunchKernelGGL(tsqr_tree_kernel, dim3(batch), dim3(TS_NT), 0, s, M, ldm, sM, c0, w, h1, r1a,
                       r2a, P, V, ldv, sV, vr2, sc.Tloc, sc.Rstack, sc.Qtop, sc.Z, sc.U, sc.L,
                       sc.S, sc.stride, T, sT);
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
