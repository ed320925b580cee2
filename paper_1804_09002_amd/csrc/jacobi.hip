// Leaf eigensolver of Zolo-eig: cyclic Jacobi on blocks of at most 64 x 64,
// one workgroup per block, the matrix and its eigenvector basis resident in LDS.
//
// A sweep visits all n(n-1)/2 pairs in n-1 rounds of n/2 disjoint pairs
// (round-robin ordering: index 0 fixed, the others rotate); the rotations of a
// round are independent, so each round is one parallel column update, one
// parallel row update and one update of V, separated by barriers.  Rotation
// (p, q): tau = (a_qq - a_pp) / (2 a_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
// c = 1/sqrt(1 + t^2), s = t c; A <- J^T A J annihilates a_pq.  Sweeps stop
// when the off-diagonal Frobenius norm is below 1e-17 ||A||_F or after 40 sweeps.
#include <cmath>

#include "zcsd_eig.h"
#include "zcsd_internal.h"

namespace zcsd {

constexpr int JB = 64;
constexpr int JNT = 256;

__global__ __launch_bounds__(JNT) void jacobi_kernel(const int* __restrict__ sizes, const double* A,
                                                     long long lda, long long sA, double* V,
                                                     long long ldv, long long sV, double* lam) {
  __shared__ double S[JB][JB + 1];
  __shared__ double Q[JB][JB + 1];
  __shared__ double cs[JB / 2][2];
  __shared__ int pq[JB / 2][2];
  __shared__ double red[JNT / 64];
  __shared__ double red2[JNT / 64];
  __shared__ int done;
  const int b = blockIdx.x;
  const int n = sizes[b];
  const int tid = threadIdx.x;
  A += (long long)b * sA;
  V += (long long)b * sV;
  lam += (long long)b * JB;
  if (n <= 0) return;
  {
    // all loads of a thread in flight at once, then the LDS stores
    constexpr int NL = JB * JB / JNT;
    double v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + JNT * q, i = e % n, j = e / n;
      v[q] = (e < n * n) ? 0.5 * (A[i + (long long)j * lda] + A[j + (long long)i * lda]) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int e = tid + JNT * q, i = e % n, j = e / n;
      if (e < n * n) {
        S[i][j] = v[q];
        Q[i][j] = (i == j) ? 1.0 : 0.0;
      }
    }
  }
  __syncthreads();
  const int m = (n % 2) ? n + 1 : n;  // players; index n is a dummy when n is odd
  for (int sweep = 0; sweep < 40; ++sweep) {
    // convergence test
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += JNT) {
      const int i = e % n, j = e / n;
      const double v = S[i][j];
      tot += v * v;
      if (i != j) off += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      tot += __shfl_xor(tot, o, 64);
    }
    if ((tid & 63) == 0) {
      red[tid >> 6] = off;
      red2[tid >> 6] = tot;
    }
    __syncthreads();
    if (tid == 0) {
      double o2 = 0.0, t2 = 0.0;
      for (int q = 0; q < JNT / 64; ++q) {
        o2 += red[q];
        t2 += red2[q];
      }
      done = (o2 <= 1e-33 * t2) ? 1 : 0;
    }
    __syncthreads();
    if (done) break;
    for (int rnd = 0; rnd < m - 1; ++rnd) {
      if (tid < m / 2) {
        auto idx = [&](int i) { return i == 0 ? 0 : ((i - 1 + rnd) % (m - 1)) + 1; };
        int p = idx(tid), q = idx(m - 1 - tid);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = S[p][q];
          if (apq != 0.0) {
            const double tau = (S[q][q] - S[p][p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        } else {
          q = p;  // dummy pair: no rotation
        }
        pq[tid][0] = p;
        pq[tid][1] = q;
        cs[tid][0] = c;
        cs[tid][1] = s;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int e = tid; e < (m / 2) * n; e += JNT) {
        const int k = e / n, i = e % n;
        const int p = pq[k][0], q = pq[k][1];
        if (p == q) continue;
        const double c = cs[k][0], s = cs[k][1];
        const double ap = S[i][p], aq = S[i][q];
        S[i][p] = c * ap - s * aq;
        S[i][q] = s * ap + c * aq;
        const double vp = Q[i][p], vq = Q[i][q];
        Q[i][p] = c * vp - s * vq;
        Q[i][q] = s * vp + c * vq;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = tid; e < (m / 2) * n; e += JNT) {
        const int k = e / n, j = e % n;
        const int p = pq[k][0], q = pq[k][1];
        if (p == q) continue;
        const double c = cs[k][0], s = cs[k][1];
        const double ap = S[p][j], aq = S[q][j];
        S[p][j] = c * ap - s * aq;
        S[q][j] = s * ap + c * aq;
      }
      __syncthreads();
      if (tid < m / 2) {
        const int p = pq[tid][0], q = pq[tid][1];
        if (p != q) {
          S[p][q] = 0.0;
          S[q][p] = 0.0;
        }
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < n * n; e += JNT) {
    const int i = e % n, j = e / n;
    V[i + (long long)j * ldv] = Q[i][j];
  }
  for (int i = tid; i < n; i += JNT) lam[i] = S[i][i];
}

void jacobi_batched(int nblk, const int* d_sizes, const double* A, long long lda, long long sA,
                    double* V, long long ldv, long long sV, double* d_lam, hipStream_t s) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(jacobi_kernel, dim3(nblk), dim3(JNT), 0, s, d_sizes, A, lda, sA, V, ldv, sV,
                     d_lam);
  ZCSD_CHECK_LAUNCH();
}

}  // namespace zcsd
