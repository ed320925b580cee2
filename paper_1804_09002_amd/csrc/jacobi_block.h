// The cyclic Jacobi solve of one block of at most 64 x 64 by one workgroup,
// shared by the leaf kernel of Zolo-eig and the one-workgroup CSD.
#pragma once
#include <hip/hip_runtime.h>

namespace zcsd {

// Cyclic Jacobi on a block of at most 64 x 64 by one workgroup, the matrix and
// its eigenvector basis resident in LDS.
//
// A sweep visits all n(n-1)/2 pairs in n-1 rounds of n/2 disjoint pairs
// (round-robin ordering: index 0 fixed, the others rotate); the rotations of a
// round are independent, so each round is one parallel column update, one
// parallel row update and one update of V, separated by barriers.  Rotation
// (p, q): tau = (a_qq - a_pp) / (2 a_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
// c = 1/sqrt(1 + t^2), s = t c; A <- J^T A J annihilates a_pq.  A rotation is
// skipped when |a_pq| <= u ||A||_F / n (dropping every such entry changes A by
// at most u ||A||_F), and the sweeps stop after one that rotated nothing (or
// after 40 sweeps); a round that rotates no pair skips its update.
//
// Every rotation applied to the basis adds rounding to it, and each column
// takes n - 1 of them per sweep, so the accumulated basis X is orthonormal
// only to about 2 n u (150 u at n = 64).  One step of the FP64 refinement of
// Ogita & Aishima (2018) in LDS then restores both orthogonality and the
// diagonalisation: with R = I - X^T X, G = X^T A X (symmetrised) and Rayleigh
// quotients l_i = G_ii / (1 - R_ii),
//     F_ij = (G_ij + l_j R_ij) / (l_j - l_i)   for |l_j - l_i| > delta,
//     F_ij = R_ij / 2                           otherwise (and on the diagonal),
//     X <- X + X F,
// so that F + F^T = R and X^T X = I to second order.  Pairs closer than
// delta = 1e-6 ||A||_F stay as Jacobi left them (their eigenvectors are
// determined only to u ||A|| / gap, and a correction divided by such a gap
// would bring rounding of G back at second order); they are orthogonalised.
// the leaf blocks of Zolo-eig: at most 64, one workgroup of 256 threads
constexpr int kLeafMax = 64;
constexpr int kLeafThreads = 256;

// LDS of one block solve (blocks of at most JB, workgroups of JNT threads)
template <int JB, int JNT>
struct JacobiShared {
  // the matrix in two buffers: a round reads one and writes J^T S J into the other
  double Sbuf[2][JB][JB + 1];
  double Q[JB][JB + 1];
  double cs[JB / 2][2];
  int pq[JB / 2][2];
  // per index i of a round: row/column i of J^T S J is al[i] (row/column i) +
  // be[i] (row/column pt[i]) of S (al = 1, be = 0 for an index not rotated)
  double al[JB], be[JB];
  int pt[JB];
  double red2[JNT / 64];
  double lt[JB];
  int rotated;
  // whether round r rotates any pair, in rround[r % 2]
  int rround[2];
};

// Eigenpairs of the symmetric part of the n x n block A (1 <= n <= JB, ld lda)
// by the workgroup of JNT threads that calls it (every thread, uniformly):
// V (n x n, ld ldv) and lam (n).  A, V and lam may be global or LDS.
template <int JB, int JNT>
__device__ inline void jacobi_block(int n, const double* A, long long lda, double* V, long long ldv,
                                    double* lam, JacobiShared<JB, JNT>& sh) {
  double(*Sbuf)[JB][JB + 1] = sh.Sbuf;
  double(*Q)[JB + 1] = sh.Q;
  double(*cs)[2] = sh.cs;
  int(*pq)[2] = sh.pq;
  double* al = sh.al;
  double* be = sh.be;
  int* pt = sh.pt;
  double* red2 = sh.red2;
  double* lt = sh.lt;
  int& rotated = sh.rotated;
  const int tid = threadIdx.x;
  // element e = tid + JNT q of the n x n block: row e % n, column e / n
  constexpr int NL = JB * JB / JNT;
  int cur = 0;
  double(*S)[JB + 1] = Sbuf[0];
  // symmetrised input into S (all loads of a thread in flight at once, then
  // the LDS stores); with_basis also resets Q to I
  auto load_input = [&](bool with_basis) {
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
        if (with_basis) Q[i][j] = (i == j) ? 1.0 : 0.0;
      }
    }
  };
  load_input(true);
  __syncthreads();
  // ||A||_F^2 (the rotation threshold and the refinement's cluster gap)
  {
    double tot = 0.0;
    for (int e = tid; e < n * n; e += JNT) {
      const double v = S[e % n][e / n];
      tot += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
    if ((tid & 63) == 0) red2[tid >> 6] = tot;
    __syncthreads();
  }
  double afro = 0.0;
  for (int q = 0; q < JNT / 64; ++q) afro += red2[q];
  afro = sqrt(afro);
  const double thr = 0x1p-53 * afro / n;
  const int m = (n % 2) ? n + 1 : n;  // players; index n is a dummy when n is odd
  // a round's updates: thread tid takes row ri = tid % RB of the columns
  // rj0 + CS q and of the pairs rj0 + CS q, RB the smallest of 16, 32, 64
  // that holds n (every thread busy for small n)
  const int RB = (n <= 16) ? 16 : ((n <= 32) ? 32 : 64);
  const int CS = JNT / RB;
  const int ri = tid & (RB - 1), rj0 = tid / RB;
  // iterations that cover JB columns and JB / 2 pairs at the smallest stride
  constexpr int RBMAX = (JB <= 16) ? 16 : ((JB <= 32) ? 32 : 64);
  constexpr int CSMIN = JNT / RBMAX;
  constexpr int NQC = (JB + CSMIN - 1) / CSMIN, NQP = (JB / 2 + CSMIN - 1) / CSMIN;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) {
      rotated = 0;
      sh.rround[0] = 0;
    }
    __syncthreads();
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
        const int q0 = q;
        if (q < n && fabs(S[p][q]) > thr) {
          const double apq = S[p][q];
          const double tau = (S[q][q] - S[p][p]) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          rotated = 1;
          sh.rround[rnd & 1] = 1;
        } else {
          q = p;  // dummy pair or an entry below the threshold: no rotation
        }
        pq[tid][0] = p;
        pq[tid][1] = q;
        cs[tid][0] = c;
        cs[tid][1] = s;
        // new column p = c col_p - s col_q, new column q = s col_p + c col_q
        // (rows alike); an index without a rotation keeps its row and column
        if (p != q) {
          al[p] = c; be[p] = -s; pt[p] = q;
          al[q] = c; be[q] = s; pt[q] = p;
        } else {
          al[p] = 1.0; be[p] = 0.0; pt[p] = p;
          if (q0 < n) {
            al[q0] = 1.0; be[q0] = 0.0; pt[q0] = q0;
          }
        }
      }
      __syncthreads();
      // a round that rotates nothing leaves S and V as they are (its update
      // would copy S unchanged into the other buffer): skipped; the flag of
      // the next round is cleared here, after every thread has read it in
      // the round before
      const bool any = sh.rround[rnd & 1] != 0;
      if (tid == 0) sh.rround[(rnd + 1) & 1] = 0;
      // S' = J^T S J into the other buffer (a column combination, then the
      // row combination of the two columns: the arithmetic of applying J on
      // the right, then J^T on the left), the rotated pairs' entries set to
      // zero; V <- V J in place (each pair's two columns by one thread)
      // (the row's rotation is read once)
      if (any && ri < n) {
        double(*Sn)[JB + 1] = Sbuf[cur ^ 1];
        const int pi = pt[ri];
        const double ai = al[ri], bi = be[ri];
#pragma unroll
        for (int qq = 0; qq < NQC; ++qq) {
          const int j = rj0 + CS * qq;
          if (j < n) {
            const int pj = pt[j];
            const double aj = al[j], bj = be[j];
            const double t1 = aj * S[ri][j] + bj * S[ri][pj];
            const double t2 = aj * S[pi][j] + bj * S[pi][pj];
            Sn[ri][j] = (pi == j && pi != ri) ? 0.0 : ai * t1 + bi * t2;
          }
        }
#pragma unroll
        for (int qq = 0; qq < NQP; ++qq) {
          const int k = rj0 + CS * qq;
          if (k < m / 2) {
            const int p = pq[k][0], q = pq[k][1];
            if (p != q) {
              const double c = cs[k][0], s = cs[k][1];
              const double vp = Q[ri][p], vq = Q[ri][q];
              Q[ri][p] = c * vp - s * vq;
              Q[ri][q] = s * vp + c * vq;
            }
          }
        }
      }
      __syncthreads();
      if (any) {
        cur ^= 1;
        S = Sbuf[cur];
      }
    }
    if (!rotated) break;
    __syncthreads();  // every thread has read `rotated` before it is reset
  }

  // --- one refinement step on the basis X = Q (Ogita & Aishima) -----------
  __syncthreads();
  load_input(false);  // S <- A
  __syncthreads();
  double x[NL], g[NL], r[NL];
  // T = A X into registers, then into S
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + JNT * q, i = e % n, j = e / n;
    double acc = 0.0;
    if (e < n * n)
      for (int k = 0; k < n; ++k) acc += S[i][k] * Q[k][j];
    x[q] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + JNT * q;
    if (e < n * n) S[e % n][e / n] = x[q];
  }
  __syncthreads();
  // G = X^T T and R = I - X^T X (the products of R_ij and R_ji are the same
  // numbers summed in the same order, so R is exactly symmetric)
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + JNT * q, i = e % n, j = e / n;
    double ag = 0.0, ar = 0.0;
    if (e < n * n)
      for (int k = 0; k < n; ++k) {
        const double xki = Q[k][i];
        ag += xki * S[k][j];
        ar += xki * Q[k][j];
      }
    g[q] = ag;
    r[q] = (i == j ? 1.0 : 0.0) - ar;
  }
  __syncthreads();
  // G symmetrised through LDS; Rayleigh quotients from its diagonal
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + JNT * q;
    if (e < n * n) S[e % n][e / n] = g[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + JNT * q, i = e % n, j = e / n;
    if (e < n * n) {
      g[q] = 0.5 * (g[q] + S[j][i]);
      if (i == j) lt[i] = g[q] / (1.0 - r[q]);
    }
  }
  __syncthreads();
  // F into S
  const double delta = 1e-6 * afro;
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + JNT * q, i = e % n, j = e / n;
    if (e < n * n) {
      const double gap = lt[j] - lt[i];
      S[i][j] = (i != j && fabs(gap) > delta) ? (g[q] + lt[j] * r[q]) / gap : 0.5 * r[q];
    }
  }
  __syncthreads();
  // X <- X + X F
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + JNT * q, i = e % n, j = e / n;
    double acc = 0.0;
    if (e < n * n)
      for (int k = 0; k < n; ++k) acc += Q[i][k] * S[k][j];
    x[q] = (e < n * n) ? Q[i][j] + acc : 0.0;
  }
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int e = tid + JNT * q;
    if (e < n * n) V[e % n + (long long)(e / n) * ldv] = x[q];
  }
  for (int i = tid; i < n; i += JNT) lam[i] = lt[i];
}

}  // namespace zcsd
