// Tall panel factorisation for the blocked Householder QR: TSQR followed by
// reconstruction of the Householder vectors.
//
// A panel of h logical rows and w <= 32 columns is cut into P row blocks of
// TS_MB rows (the last one takes the remainder, < 2 TS_MB rows):
//   A. every block is factored in LDS by one workgroup, Q_p R_p (local
//      Householder vectors Y_p and compact-WY factor T_p);
//   B. one workgroup factors the stacked [R_1; ...; R_P] = Q_top R, forms the
//      explicit Q_top, the top w x w block Q_00 of the panel's Q, and the
//      LU factorisation Q_00 - S = L_1 U with the sign of each pivot chosen so
//      that |pivot| >= 1 (S = diag(+-1)).  Then the panel's Householder form is
//      V = [L_1; Q_rest U^{-1}], T = -U S L_1^{-T}, R = S R_tsqr
//      (Ballard, Demmel, Grigori, Jacobsen, Knight, Nguyen, "Reconstructing
//      Householder vectors from tall-skinny QR", 2015);
//   C. every block forms its rows of the explicit Q,
//      Q_p = (I - Y_p T_p Y_p^T) [Q_top,p; 0], and of V = Q U^{-1}.
// Each stage is parallel over rows; only the w x w pieces are sequential.
// The result is interchangeable with a column-by-column Householder panel
// (same R up to row signs, V unit lower trapezoidal, H = I - V T V^T).
#include <algorithm>
#include <cmath>

#include "zcsd_internal.h"
#include "zcsd_la.h"
#include "zcsd_qr_tsqr.h"

namespace zcsd {

constexpr int TS_NT = 256;
constexpr int TS_W = 32;                    // panel width handled here
constexpr int TS_LD = 2 * TS_MB + 1;        // LDS leading dimension (odd)

__device__ __forceinline__ int ts_phys(int i, int h1, int r1a, int r2a) {
  return i < h1 ? r1a + i : r2a + (i - h1);
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < TS_NT / 64; ++q) s += red[q];
  return s;
}

// Householder QR of A (rows x w, column-major in LDS with leading dim LD) in
// place: v's below the diagonal with implicit unit diagonal, R on and above
// (betas hold R's diagonal, A's diagonal is set to 1), T (w x w) in Ts.
// 256 threads; the dot products d_j = v^T A(:, j) use 8 threads per column.
__device__ void lds_householder(double* A, int LD, int rows, int w, double (*Ts)[TS_W + 1],
                                double* betas, double* red, double* sums) {
  const int tid = threadIdx.x;
  const int grp = tid >> 3, gl = tid & 7;  // 32 groups of 8 threads
  for (int e = tid; e < TS_W * (TS_W + 1); e += TS_NT) (&Ts[0][0])[e] = 0.0;
  for (int t = 0; t < w; ++t) {
    double* at = A + (long long)t * LD;
    double p = 0.0;
    for (int i = t + 1 + tid; i < rows; i += TS_NT) p += at[i] * at[i];
    const double sig2 = block_sum(p, red);
    const double alpha = at[t];
    double tau, beta, scal;
    if (sig2 == 0.0) {
      tau = 0.0;
      beta = alpha;
      scal = 1.0;
    } else {
      const double nrm = sqrt(alpha * alpha + sig2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    __syncthreads();
    for (int i = t + 1 + tid; i < rows; i += TS_NT) at[i] *= scal;
    if (tid == 0) {
      at[t] = 1.0;
      betas[t] = beta;
    }
    __syncthreads();
    // d_j = sum_{i >= t} v_i A(i, j), j = grp (group of 8 threads per column)
    {
      const int j = grp;
      double s = 0.0;
      if (j < w && j != t) {
        const double* aj = A + (long long)j * LD;
        for (int i = t + gl; i < rows; i += 8) s += at[i] * aj[i];
      }
      s += __shfl_xor(s, 4, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 1, 64);
      if (gl == 0) sums[j] = s;
    }
    __syncthreads();
    if (tid < t) {
      double s = 0.0;
      for (int q = tid; q < t; ++q) s += Ts[tid][q] * sums[q];
      Ts[tid][t] = -tau * s;
    }
    if (tid == 0) Ts[t][t] = tau;
    const int nup = w - t - 1;
    if (nup > 0 && tau != 0.0) {
      const int len = rows - t;
      for (int e = tid; e < len * nup; e += TS_NT) {
        const int i = t + e % len, j = t + 1 + e / len;
        A[i + (long long)j * LD] -= tau * sums[j] * at[i];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// A: local QR of every row block
__global__ __launch_bounds__(TS_NT) void tsqr_local_kernel(
    const double* M, long long ldm, long long sM, int c0, int w, int h1, int r1a, int r2a, int h,
    int P, double* V, long long ldv, long long sV, double* Tloc, double* Rstack, long long sScr) {
  __shared__ double A[TS_W * TS_LD];
  __shared__ double Ts[TS_W][TS_W + 1];
  __shared__ double betas[TS_W];
  __shared__ double red[TS_NT / 64];
  __shared__ double sums[TS_W];
  const int p = blockIdx.x;
  const long long b = blockIdx.y;
  M += b * sM;
  V += b * sV;
  const int i0 = p * TS_MB;
  const int rows = (p == P - 1) ? h - i0 : TS_MB;
  const int tid = threadIdx.x;
  for (int e = tid; e < rows * w; e += TS_NT) {
    const int i = e % rows, j = e / rows;
    A[i + j * TS_LD] = M[ts_phys(i0 + i, h1, r1a, r2a) + (long long)(c0 + j) * ldm];
  }
  __syncthreads();
  lds_householder(A, TS_LD, rows, w, Ts, betas, red, sums);
  // outputs: Y_p (unit lower trapezoidal) into V's rows, T_p, R_p (upper w x w)
  for (int e = tid; e < rows * w; e += TS_NT) {
    const int i = e % rows, j = e / rows;
    double y;
    if (i < j) y = 0.0;
    else if (i == j) y = 1.0;
    else y = A[i + j * TS_LD];
    V[(i0 + i) + (long long)j * ldv] = y;
  }
  double* Tp = Tloc + b * sScr + (long long)p * TS_W * TS_W;
  double* Rp = Rstack + b * sScr;
  const int ldr = P * TS_W;
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e % TS_W, j = e / TS_W;
    Tp[e] = (i < w && j < w) ? Ts[i][j] : 0.0;
    double r = 0.0;
    if (i < w && j < w && i <= j) r = (i == j) ? betas[i] : A[i + j * TS_LD];
    if (i < w && j < w) Rp[(p * w + i) + (long long)j * ldr] = r;
  }
}

// B: QR of the stacked R factors, explicit Q_top, reconstruction pieces.
// LDS: the stacked matrix (dead once Q_top is formed, then reused for the
// w x w work arrays), T_top, Z = T_top Y_top(0:w,:)^T and R_tsqr.
__global__ __launch_bounds__(TS_NT) void tsqr_tree_kernel(
    double* M, long long ldm, long long sM, int c0, int w, int h1, int r1a, int r2a, int P,
    const double* V, long long ldv, long long sV, const double* Tloc, const double* Rstack,
    double* Qtop, double* Uo, double* Lo, double* So, long long sScr, double* Tfin, long long sT) {
  constexpr int W1 = TS_W + 1;
  __shared__ double A[TS_W * TS_LD];
  __shared__ double Ts[TS_W][W1];
  __shared__ double Z[TS_W][W1];
  __shared__ double Rf[TS_W][W1];
  __shared__ double betas[TS_W];
  __shared__ double red[TS_NT / 64];
  __shared__ double sums[TS_W];
  __shared__ double sg[TS_W];
  __shared__ double piv_sh;
  const long long b = blockIdx.x;
  M += b * sM;
  V += b * sV;
  Tloc += b * sScr;
  Rstack += b * sScr;
  Qtop += b * sScr;
  Uo += b * sScr;
  Lo += b * sScr;
  So += b * sScr;
  Tfin += b * sT;
  const int tid = threadIdx.x;
  const int rows = P * w;
  const int ldr = P * TS_W;
  for (int e = tid; e < rows * w; e += TS_NT) {
    const int i = e % rows, j = e / rows;
    A[i + j * TS_LD] = Rstack[i + (long long)j * ldr];
  }
  __syncthreads();
  lds_householder(A, TS_LD, rows, w, Ts, betas, red, sums);
  // R_tsqr (upper w x w) and Z = T_top Y_top(0:w, :)^T, Y_top unit lower
  for (int e = tid; e < w * w; e += TS_NT) {
    const int i = e % w, j = e / w;
    Rf[i][j] = (i < j) ? A[i + j * TS_LD] : ((i == j) ? betas[i] : 0.0);
    double s = 0.0;
    for (int q = i; q <= j && q < w; ++q) {
      const double y = (j == q) ? 1.0 : A[j + q * TS_LD];  // Y(j, q), j >= q
      s += Ts[i][q] * y;
    }
    Z[i][j] = s;
  }
  __syncthreads();
  // Q_top = [I; 0] - Y_top Z  (rows x w) -> global
  for (int e = tid; e < rows * w; e += TS_NT) {
    const int i = e % rows, j = e / rows;
    double s = (i == j) ? 1.0 : 0.0;
    const int qmax = min(i, w - 1);
    for (int q = 0; q <= qmax; ++q) {
      const double y = (i == q) ? 1.0 : A[i + q * TS_LD];
      s -= y * Z[q][j];
    }
    Qtop[i + (long long)j * ldr] = s;
  }
  __syncthreads();  // A is dead from here on: reuse it for w x w arrays
  double* Q0 = A;                   // Q_00, then its LU in place
  double* Y0 = A + TS_W * W1;       // Y_0(0:w, 0:w) of block 0 (unit lower)
  double* Li = A + 2 * TS_W * W1;   // temporaries, then L1^{-T}
  double* X2 = A + 3 * TS_W * W1;
#define S2(p, i, j) p[(i) * W1 + (j)]
  for (int e = tid; e < w * w; e += TS_NT) {
    const int i = e % w, j = e / w;
    S2(Q0, i, j) = Qtop[i + (long long)j * ldr];
    S2(Y0, i, j) = (i < j) ? 0.0 : ((i == j) ? 1.0 : V[i + (long long)j * ldv]);
  }
  __syncthreads();
  // Q_00 = Q_top,0 - Y0 T_0 (Y0^T Q_top,0)
  const double* T0 = Tloc;
  for (int e = tid; e < w * w; e += TS_NT) {
    const int i = e % w, j = e / w;
    double s = 0.0;
    for (int q = i; q < w; ++q) s += S2(Y0, q, i) * S2(Q0, q, j);
    S2(X2, i, j) = s;
  }
  __syncthreads();
  for (int e = tid; e < w * w; e += TS_NT) {
    const int i = e % w, j = e / w;
    double s = 0.0;
    for (int q = i; q < w; ++q) s += T0[i + q * TS_W] * S2(X2, q, j);
    S2(Li, i, j) = s;
  }
  __syncthreads();
  for (int e = tid; e < w * w; e += TS_NT) {
    const int i = e % w, j = e / w;
    double s = 0.0;
    for (int q = 0; q <= i; ++q) s += S2(Y0, i, q) * S2(Li, q, j);
    S2(X2, i, j) = S2(Q0, i, j) - s;
  }
  __syncthreads();
  for (int e = tid; e < w * w; e += TS_NT) {
    const int i = e % w, j = e / w;
    S2(Q0, i, j) = S2(X2, i, j);
  }
  __syncthreads();
  // LU of Q_00 - S with the pivot sign chosen so that |pivot| >= 1
  for (int k = 0; k < w; ++k) {
    if (tid == 0) {
      const double sk = (S2(Q0, k, k) >= 0.0) ? -1.0 : 1.0;
      sg[k] = sk;
      S2(Q0, k, k) -= sk;
      piv_sh = S2(Q0, k, k);
    }
    __syncthreads();
    const int m = w - k - 1;
    if (tid < m) S2(Q0, k + 1 + tid, k) /= piv_sh;
    __syncthreads();
    for (int e = tid; e < m * m; e += TS_NT) {
      const int i = k + 1 + e % m, j = k + 1 + e / m;
      S2(Q0, i, j) -= S2(Q0, i, k) * S2(Q0, k, j);
    }
    __syncthreads();
  }
  // Li = L1^{-T}: thread j computes column j of L1^{-1} (forward substitution)
  if (tid < w) {
    const int j = tid;
    for (int i = 0; i < w; ++i) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int q = j; q < i; ++q) s -= S2(Q0, i, q) * S2(Li, j, q);
      S2(Li, j, i) = (i < j) ? 0.0 : s;  // L1^{-T}(j, i) = L1^{-1}(i, j)
    }
  }
  __syncthreads();
  // T = -U S L1^{-T} (upper), U = upper part of the LU
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e % TS_W, j = e / TS_W;
    double s = 0.0;
    if (i < w && j < w && i <= j)
      for (int q = i; q <= j; ++q) s += S2(Q0, i, q) * sg[q] * S2(Li, q, j);
    Tfin[i + (long long)j * TS_W] = -s;
  }
  // R = S R_tsqr into the matrix (top w logical rows = segment 1), zeros below the diagonal
  for (int e = tid; e < w * w; e += TS_NT) {
    const int i = e % w, j = e / w;
    M[ts_phys(i, h1, r1a, r2a) + (long long)(c0 + j) * ldm] = (i <= j) ? sg[i] * Rf[i][j] : 0.0;
  }
  // U, L1, S for the row expansion
  for (int e = tid; e < w * w; e += TS_NT) {
    const int i = e % w, j = e / w;
    Uo[i + j * TS_W] = (i <= j) ? S2(Q0, i, j) : 0.0;
    Lo[i + j * TS_W] = (i > j) ? S2(Q0, i, j) : ((i == j) ? 1.0 : 0.0);
  }
  if (tid < w) So[tid] = sg[tid];
#undef S2
}

// C: rows of Q and of V = Q U^{-1}; zero the annihilated panel entries
__global__ __launch_bounds__(TS_NT) void tsqr_expand_kernel(
    double* M, long long ldm, long long sM, int c0, int w, int h1, int r1a, int r2a, int h, int P,
    double* V, long long ldv, long long sV, const double* Tloc, const double* Qtop,
    const double* Uo, const double* Lo, long long sScr) {
  __shared__ double M1[TS_W][TS_W + 1];
  __shared__ double M2[TS_W][TS_W + 1];
  __shared__ double Us[TS_W][TS_W + 1];
  __shared__ double Qt[TS_W][TS_W + 1];
  __shared__ double Qr[TS_W][TS_NT + 1];
  const int p = blockIdx.x;
  const long long b = blockIdx.y;
  M += b * sM;
  V += b * sV;
  Tloc += b * sScr;
  Qtop += b * sScr;
  Uo += b * sScr;
  Lo += b * sScr;
  const int tid = threadIdx.x;
  const int i0 = p * TS_MB;
  const int rows = (p == P - 1) ? h - i0 : TS_MB;
  const int ldr = P * TS_W;
  const double* Tp = Tloc + (long long)p * TS_W * TS_W;
  for (int e = tid; e < w * w; e += TS_NT) {
    const int i = e % w, j = e / w;
    Qt[i][j] = Qtop[(p * w + i) + (long long)j * ldr];
    Us[i][j] = Uo[i + j * TS_W];
  }
  __syncthreads();
  // M1 = Y_p(0:w, :)^T Qt_p,  Y_p unit lower on its first w rows
  for (int e = tid; e < w * w; e += TS_NT) {
    const int i = e % w, j = e / w;
    double s = 0.0;
    for (int q = i; q < w; ++q) s += ((q == i) ? 1.0 : V[(i0 + q) + (long long)i * ldv]) * Qt[q][j];
    M1[i][j] = s;
  }
  __syncthreads();
  for (int e = tid; e < TS_W * TS_W; e += TS_NT) {
    const int i = e % TS_W, j = e / TS_W;
    double s = 0.0;  // rows/columns beyond w stay exactly zero (they multiply y_k = 0)
    if (i < w && j < w)
      for (int q = i; q < w; ++q) s += Tp[i + q * TS_W] * M1[q][j];
    M2[i][j] = s;
  }
  __syncthreads();
  // row by row: q = [Qt_p; 0](i, :) - Y_p(i, :) M2, then v = q U^{-1}; in place over Y_p.
  // y lives in registers (fully unrolled over the 32 columns), q in LDS (one column of
  // Qr per panel column, one entry per thread).
  for (int i = tid; i < rows; i += TS_NT) {
    const int gi = i0 + i;
    double y[TS_W];
#pragma unroll
    for (int k = 0; k < TS_W; ++k) y[k] = (k < w) ? V[gi + (long long)k * ldv] : 0.0;
    for (int j = 0; j < w; ++j) {
      double s = (i < w) ? Qt[i][j] : 0.0;
#pragma unroll
      for (int k = 0; k < TS_W; ++k) s -= y[k] * M2[k][j];
      Qr[j][tid] = s;
    }
    if (p == 0 && i < w) {
      for (int j = 0; j < w; ++j) V[gi + (long long)j * ldv] = Lo[i + j * TS_W];
    } else {
      // v U = q, U upper: v_j = (q_j - sum_{k<j} v_k U(k, j)) / U(j, j), v overwrites q
      for (int j = 0; j < w; ++j) {
        double s = Qr[j][tid];
        for (int k = 0; k < j; ++k) s -= Qr[k][tid] * Us[k][j];
        Qr[j][tid] = s / Us[j][j];
      }
      for (int j = 0; j < w; ++j) V[gi + (long long)j * ldv] = Qr[j][tid];
    }
    if (gi >= w) {
      const long long pr = ts_phys(gi, h1, r1a, r2a);
      for (int j = 0; j < w; ++j) M[pr + (long long)(c0 + j) * ldm] = 0.0;
    }
  }
}

bool tsqr_panel_fits(int h, int w) { return w <= TS_W && w >= 1 && h >= w && h < (TS_PMAX + 1) * TS_MB; }

void tsqr_panel(int batch, double* M, long long ldm, long long sM, int c0, int w, int r1a, int r1b,
                int r2a, int r2b, double* V, long long ldv, long long sV, double* T, long long sT,
                const TsqrScratch& sc, hipStream_t s) {
  const int h1 = r1b - r1a, h2 = r2b - r2a, h = h1 + h2;
  const int P = std::max(1, h / TS_MB);
  if (!tsqr_panel_fits(h, w) || P > TS_PMAX) throw ArgError("tsqr_panel: panel too tall");
  hipLaunchKernelGGL(tsqr_local_kernel, dim3(P, batch), dim3(TS_NT), 0, s, M, ldm, sM, c0, w, h1,
                     r1a, r2a, h, P, V, ldv, sV, sc.Tloc, sc.Rstack, sc.stride);
  ZCSD_CHECK_LAUNCH();
  hipLaunchKernelGGL(tsqr_tree_kernel, dim3(batch), dim3(TS_NT), 0, s, M, ldm, sM, c0, w, h1, r1a,
                     r2a, P, V, ldv, sV, sc.Tloc, sc.Rstack, sc.Qtop, sc.U, sc.L, sc.S, sc.stride,
                     T, sT);
  ZCSD_CHECK_LAUNCH();
  hipLaunchKernelGGL(tsqr_expand_kernel, dim3(P, batch), dim3(TS_NT), 0, s, M, ldm, sM, c0, w, h1,
                     r1a, r2a, h, P, V, ldv, sV, sc.Tloc, sc.Qtop, sc.U, sc.L, sc.stride);
  ZCSD_CHECK_LAUNCH();
}

TsqrScratch tsqr_scratch_alloc(Arena& ar, int batch) {
  TsqrScratch sc;
  const long long per_R = (long long)TS_PMAX * TS_W * TS_W;  // Rstack, Qtop: (P w) x w
  sc.stride = 4 * per_R + 3 * TS_W * TS_W + TS_W;
  double* base = ar.dalloc((size_t)batch * sc.stride);
  sc.Rstack = base;
  sc.Qtop = base + per_R;
  sc.Tloc = base + 2 * per_R;  // P blocks of w x w
  sc.U = base + 4 * per_R;
  sc.L = sc.U + TS_W * TS_W;
  sc.S = sc.L + TS_W * TS_W;
  return sc;
}

}  // namespace zcsd
