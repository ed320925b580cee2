// Cholesky factorisation with its inverse factor, and upper-triangular inverse.
//
// Zolo-pd's Cholesky form (Sec. 5) needs X (X^T X + c I)^{-1} = X R^{-1} R^{-T}
// with R^T R = X^T X + c I.  chol_inv_batched returns R and R^{-1} together by
// the block recursion
//     R11 = chol(A11),  R12 = R11^{-T} A12,  R22 = chol(A22 - R12^T R12),
//     (R^{-1})12 = -R11^{-1} R12 R22^{-1},
// so the triangular solves become MFMA GEMMs; blocks of at most CH_BASE are
// factored in LDS by one workgroup and inverted there by 16 x 16 MFMA blocks.
//
// trtri_upper_batched inverts an upper-triangular R: all diagonal blocks of
// size CH_BASE are inverted at once, then neighbouring blocks are merged level
// by level, (R^{-1})_{AB} = -R_A^{-1} R_{AB} R_B^{-1}, every pair of a level in
// one batched GEMM.
#include <algorithm>
#include <cmath>

#include "zcsd_internal.h"
#include "zcsd_la.h"

namespace zcsd {

constexpr int CH_BASE = 64;
constexpr int CH_NT = 256;
constexpr int CH_LD = CH_BASE + 1;

typedef double d4 __attribute__((ext_vector_type(4)));

// 16 x 16 block of X(i0:i0+16, kx0:kx0+K) * Y(ky0:ky0+K, j0:j0+16) on the FP64
// matrix cores, both operands in LDS ([row][col]).  v_mfma_f64_16x16x4f64 takes
// a[i][k] from lane i + 16k and b[k][j] from lane j + 16k and leaves d[i][j] in
// item i / 4 of lane j + 16 (i % 4); fed with Y^T as "a" and X^T as "b" it
// holds the transposed block, so lane l item v is C[l % 16][4 v + l / 16].
template <int K>
__device__ __forceinline__ d4 lds_mm16(const double (*X)[CH_LD], int i0, int kx0,
                                       const double (*Y)[CH_LD], int ky0, int j0) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < K; kk += 4) {
    const double fa = X[i0 + lr][kx0 + kk + lk];
    const double fb = Y[ky0 + kk + lk][j0 + lr];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fb, fa, acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ void lds_put16(double (*C)[CH_LD], int i0, int j0, d4 acc, double scale) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 4; ++v) C[i0 + (lane & 15)][j0 + 4 * v + (lane >> 4)] = scale * acc[v];
}

// Inverse of the 64 x 64 upper-triangular U held in LDS (exact zeros below the
// diagonal, identity beyond the problem's size) into Ui, by all 256 threads:
// the four 16 x 16 diagonal blocks by back substitution (one column per
// thread), then two merge levels (Ui)_AB = -Ui_A (U_AB Ui_B) as 16 x 16 MFMA
// blocks (pairs of 16-blocks, then the two 32-blocks).  dinv[i] = 1 / U[i][i]
// on entry; Xs is 32 x 32 scratch.  Ends with a barrier.
__device__ void lds_upper_inverse64(const double (*U)[CH_LD], double (*Ui)[CH_LD],
                                    const double* dinv, double (*Xs)[CH_LD]) {
  const int tid = threadIdx.x, wave = tid >> 6;
  for (int e = tid; e < CH_BASE * CH_BASE; e += CH_NT) Ui[e & 63][e >> 6] = 0.0;
  __syncthreads();
  if (tid < CH_BASE) {
    const int o = tid & ~15, c = tid & 15;
    double x[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double s = 0.0;
#pragma unroll
      for (int p = i + 1; p < 16; ++p) s = fma(U[o + i][o + p], x[p], s);
      x[i] = (i > c) ? 0.0 : ((i == c) ? dinv[o + c] : -s * dinv[o + i]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i <= c) Ui[o + i][o + c] = x[i];
  }
  __syncthreads();
  // pairs (A, B) = ([o, o+16), [o+16, o+32)), o = 32 wave, on waves 0 and 1
  if (wave < 2) {
    const int o = 32 * wave;
    lds_put16(Xs, 16 * wave, 0, lds_mm16<16>(U, o, o + 16, Ui, o + 16, o + 16), 1.0);
  }
  __syncthreads();
  if (wave < 2) {
    const int o = 32 * wave;
    lds_put16(Ui, o, o + 16, lds_mm16<16>(Ui, o, o, Xs, 16 * wave, 0), -1.0);
  }
  __syncthreads();
  {  // A = [0, 32), B = [32, 64); wave owns the 16 x 16 tile (ti, tj) of the 32 x 32 block
    const int ti = wave & 1, tj = wave >> 1;
    const d4 xab = lds_mm16<32>(U, 16 * ti, 32, Ui, 32, 32 + 16 * tj);
    lds_put16(Xs, 16 * ti, 16 * tj, xab, 1.0);
    __syncthreads();
    const d4 yab = lds_mm16<32>(Ui, 16 * ti, 0, Xs, 0, 16 * tj);
    lds_put16(Ui, 16 * ti, 32 + 16 * tj, yab, -1.0);
  }
  __syncthreads();
}

// one workgroup per problem: A (nb x nb, symmetric, upper triangle read) -> R, Ri.
// Right-looking Cholesky on the unscaled pivot rows, S22 -= s12^T s12 / s11,
// with the upper triangle in registers: thread (bi, bj) owns the 4 x 4 block
// S(4bi.., 4bj..), bi <= bj; the owners of row k + 1 publish it to LDS once
// step k has finalised it (one barrier per step, eight LDS reads per thread).
// Then R(k, :) = S(k, :) / sqrt(s_kk); a non-positive pivot is counted in
// d_flag and replaced by 1e-300.
__global__ __launch_bounds__(CH_NT) void chol_inv_base_kernel(int nb, const double* A, long long lda,
                                                              long long sA, double* R, long long ldr,
                                                              long long sR, double* Ri,
                                                              long long ldi, long long sI,
                                                              int* d_flag) {
  __shared__ double S[CH_BASE][CH_LD];
  __shared__ double Ui[CH_BASE][CH_LD];
  __shared__ double Xs[32][CH_LD];
  __shared__ double dinv[CH_BASE];
  __shared__ double prow[2][CH_BASE];
  const long long b = blockIdx.x;
  A += b * sA;
  R += b * sR;
  Ri += b * sI;
  const int tid = threadIdx.x;
  {
    // all loads of a thread in flight at once, then the LDS stores
    constexpr int NL = CH_BASE * CH_BASE / CH_NT;
    double v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + CH_NT * q, i = e & 63, j = e >> 6;
      v[q] = (i == j) ? 1.0 : 0.0;
      if (i < nb && j < nb) v[q] = (i <= j) ? A[i + (long long)j * lda] : A[j + (long long)i * lda];
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + CH_NT * q;
      S[e & 63][e >> 6] = v[q];
    }
  }
  __syncthreads();
  const int bi = tid & 15, bj = tid >> 4;
  const bool act = bi <= bj;
  double c[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) c[x][y] = S[4 * bi + x][4 * bj + y];
  if (bi == 0) {
#pragma unroll
    for (int y = 0; y < 4; ++y) prow[0][4 * bj + y] = c[0][y];
  }
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    const double* pk = prow[k & 1];
    double d = pk[k];
    if (!(d > 0.0)) d = 1e-300;
    const double inv = 1.0 / d;
    double ri[4], rj[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      ri[x] = pk[4 * bi + x] * inv;
      rj[x] = pk[4 * bj + x];
    }
    if (act) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          if (4 * bi + x > k && 4 * bj + y > k) c[x][y] = fma(-ri[x], rj[y], c[x][y]);
    }
    const int k1 = k + 1;
    if (k1 < nb && bi == (k1 >> 2)) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
        if (x == (k1 & 3)) {
#pragma unroll
          for (int y = 0; y < 4; ++y) prow[k1 & 1][4 * bj + y] = c[x][y];
        }
    }
    __syncthreads();
  }
  if (act) {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) S[4 * bi + x][4 * bj + y] = c[x][y];
  }
  __syncthreads();
  if (tid < CH_BASE) {
    double d = S[tid][tid];
    if (!(d > 0.0)) {
      if (d_flag && tid < nb) atomicAdd(d_flag, 1);
      d = 1e-300;
    }
    dinv[tid] = 1.0 / sqrt(d);
  }
  __syncthreads();
  // R = diag(1 / sqrt(s_kk)) * (upper part of S), zeros below the diagonal
  for (int e = tid; e < CH_BASE * CH_BASE; e += CH_NT) {
    const int i = e & 63, j = e >> 6;
    const double v = S[i][j];
    S[i][j] = (i < j) ? v * dinv[i] : ((i == j) ? 1.0 / dinv[i] : 0.0);
  }
  __syncthreads();
  lds_upper_inverse64(S, Ui, dinv, Xs);
  for (int e = tid; e < nb * nb; e += CH_NT) {
    const int i = e % nb, j = e / nb;
    R[i + (long long)j * ldr] = S[i][j];
    Ri[i + (long long)j * ldi] = Ui[i][j];
  }
}

// one workgroup per (problem, diagonal block)
__global__ __launch_bounds__(CH_NT) void trtri_base_kernel(int n, const double* R, long long ldr,
                                                           long long sR, double* Ri, long long ldi,
                                                           long long sI) {
  __shared__ double U[CH_BASE][CH_LD];
  __shared__ double Ui[CH_BASE][CH_LD];
  __shared__ double Xs[32][CH_LD];
  __shared__ double dinv[CH_BASE];
  const long long b = blockIdx.y;
  const int o = blockIdx.x * CH_BASE;
  const int nb = min(CH_BASE, n - o);
  R += b * sR + o + (long long)o * ldr;
  Ri += b * sI + o + (long long)o * ldi;
  const int tid = threadIdx.x;
  {
    constexpr int NL = CH_BASE * CH_BASE / CH_NT;
    double v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + CH_NT * q, i = e & 63, j = e >> 6;
      v[q] = (i == j) ? 1.0 : 0.0;
      if (i < nb && j < nb) v[q] = (i <= j) ? R[i + (long long)j * ldr] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + CH_NT * q;
      U[e & 63][e >> 6] = v[q];
    }
  }
  __syncthreads();
  if (tid < CH_BASE) dinv[tid] = 1.0 / U[tid][tid];
  __syncthreads();
  lds_upper_inverse64(U, Ui, dinv, Xs);
  for (int e = tid; e < nb * nb; e += CH_NT) {
    const int i = e % nb, j = e / nb;
    Ri[i + (long long)j * ldi] = Ui[i][j];
  }
}

// ---------------------------------------------------------------------------
static void chol_inv_rec(int batch, int n, double* A, long long lda, long long sA, double* R,
                         double* Ri, long long ld, long long s, Arena& ar, hipStream_t st) {
  if (n <= CH_BASE) {
    hipLaunchKernelGGL(chol_inv_base_kernel, dim3(batch), dim3(CH_NT), 0, st, n, A, lda, sA, R,
                       ld, s, Ri, ld, s, (int*)nullptr);
    ZCSD_CHECK_LAUNCH();
    return;
  }
  int n1 = ((n / 2 + CH_BASE - 1) / CH_BASE) * CH_BASE;
  if (n1 >= n) n1 = n - CH_BASE;
  const int n2 = n - n1;
  double* A12 = A + (long long)n1 * lda;
  double* A22 = A + n1 + (long long)n1 * lda;
  double* R12 = R + (long long)n1 * ld;
  double* R22 = R + n1 + (long long)n1 * ld;
  double* Ri12 = Ri + (long long)n1 * ld;
  double* Ri22 = Ri + n1 + (long long)n1 * ld;
  chol_inv_rec(batch, n1, A, lda, sA, R, Ri, ld, s, ar, st);
  GemmBatch g;
  g.batch = batch;
  // R12 = R11i^T A12
  g.transA = 1; g.transB = 0; g.m = n1; g.n = n2; g.k = n1;
  g.A = Ri; g.lda = ld; g.sA = s;
  g.B = A12; g.ldb = lda; g.sB = sA;
  g.C = R12; g.ldc = ld; g.sC = s;
  g.alpha = 1.0; g.beta = 0.0;
  g.tri = 2; g.kseg = n1;  // R11i^T lower triangular
  dgemm(g, st);
  // A22 <- A22 - R12^T R12
  GemmBatch h;
  h.batch = batch;
  h.transA = 1; h.transB = 0; h.m = n2; h.n = n2; h.k = n1;
  h.A = R12; h.lda = ld; h.sA = s;
  h.B = R12; h.ldb = ld; h.sB = s;
  h.C = A22; h.ldc = lda; h.sC = sA;
  h.alpha = -1.0; h.beta = 1.0;
  h.upper_only = true;  // only the upper triangle of A22 is read below
  dgemm(h, st);
  chol_inv_rec(batch, n2, A22, lda, sA, R22, Ri22, ld, s, ar, st);
  // Ri12 = -R11i (R12 R22i)
  ArenaScope scope(ar);
  double* X = ar.dalloc((size_t)batch * n1 * n2);
  GemmBatch x;
  x.batch = batch;
  x.transA = 0; x.transB = 0; x.m = n1; x.n = n2; x.k = n2;
  x.A = R12; x.lda = ld; x.sA = s;
  x.B = Ri22; x.ldb = ld; x.sB = s;
  x.C = X; x.ldc = n1; x.sC = (long long)n1 * n2;
  x.alpha = 1.0; x.beta = 0.0;
  x.tri = 4; x.kseg = n2;  // R22i upper triangular
  dgemm(x, st);
  GemmBatch y;
  y.batch = batch;
  y.transA = 0; y.transB = 0; y.m = n1; y.n = n2; y.k = n1;
  y.A = Ri; y.lda = ld; y.sA = s;
  y.B = X; y.ldb = n1; y.sB = (long long)n1 * n2;
  y.C = Ri12; y.ldc = ld; y.sC = s;
  y.alpha = -1.0; y.beta = 0.0;
  y.tri = 1; y.kseg = n1;  // R11i upper triangular
  dgemm(y, st);
}

void chol_inv_batched(int batch, int n, double* A, long long lda, long long sA, double* R,
                      double* Ri, Arena& ar, hipStream_t s) {
  if (batch <= 0 || n <= 0) return;
  const long long nn = (long long)n * n;
  // the blocks below the diagonal of R and R^{-1} are never written by the recursion
  set_identity(batch, n, n, 0.0, R, n, nn, s);
  set_identity(batch, n, n, 0.0, Ri, n, nn, s);
  chol_inv_rec(batch, n, A, lda, sA, R, Ri, n, nn, ar, s);
}

void trtri_upper_batched(int batch, int n, const double* R, long long ldr, long long sR, double* Ri,
                         long long ldi, long long sI, Arena& ar, hipStream_t s) {
  if (batch <= 0 || n <= 0) return;
  set_identity(batch, n, n, 0.0, Ri, ldi, sI, s);
  const int nblk = (n + CH_BASE - 1) / CH_BASE;
  hipLaunchKernelGGL(trtri_base_kernel, dim3(nblk, batch), dim3(CH_NT), 0, s, n, R, ldr, sR, Ri,
                     ldi, sI);
  ZCSD_CHECK_LAUNCH();
  ArenaScope scope(ar);
  for (int sz = CH_BASE; sz < n; sz *= 2) {
    // pairs (A, B) with A = [o, o + sz), B = [o + sz, min(o + 2 sz, n)), o = 2 sz p
    const int npairs_full = n / (2 * sz);
    const int rem = n - npairs_full * 2 * sz;  // leftover rows after the full pairs
    double* X = ar.dalloc((size_t)batch * (npairs_full + 1) * sz * sz);
    auto merge = [&](int o, int np, int nbB) {
      if (np <= 0 || nbB <= 0) return;
      const long long pstrideR = 2LL * sz * (ldr + 1), pstrideI = 2LL * sz * (ldi + 1);
      // X = R_AB Ri_B  (sz x nbB)
      GemmBatch g;
      g.batch = batch; g.batch2 = np;
      g.transA = 0; g.transB = 0; g.m = sz; g.n = nbB; g.k = nbB;
      g.A = R + o + (long long)(o + sz) * ldr; g.lda = ldr; g.sA = sR; g.sA2 = pstrideR;
      g.B = Ri + (o + sz) + (long long)(o + sz) * ldi; g.ldb = ldi; g.sB = sI; g.sB2 = pstrideI;
      g.C = X; g.ldc = sz; g.sC = (long long)(npairs_full + 1) * sz * sz; g.sC2 = (long long)sz * sz;
      g.alpha = 1.0; g.beta = 0.0;
      g.tri = 4; g.kseg = nbB;  // Ri_B upper triangular
      dgemm(g, s);
      // Ri_AB = -Ri_A X
      GemmBatch h;
      h.batch = batch; h.batch2 = np;
      h.transA = 0; h.transB = 0; h.m = sz; h.n = nbB; h.k = sz;
      h.A = Ri + o + (long long)o * ldi; h.lda = ldi; h.sA = sI; h.sA2 = pstrideI;
      h.B = X; h.ldb = sz; h.sB = g.sC; h.sB2 = g.sC2;
      h.C = Ri + o + (long long)(o + sz) * ldi; h.ldc = ldi; h.sC = sI; h.sC2 = pstrideI;
      h.alpha = -1.0; h.beta = 0.0;
      h.tri = 1; h.kseg = sz;  // Ri_A upper triangular
      dgemm(h, s);
    };
    merge(0, npairs_full, sz);
    if (rem > sz) merge(npairs_full * 2 * sz, 1, rem - sz);
    ar.release(scope.m);
  }
}

}  // namespace zcsd
