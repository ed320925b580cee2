// Device linear-algebra building blocks of the Zolo-csd path (internal).
#pragma once
#include "zcsd_internal.h"
#include "zcsd_qr_tsqr.h"

namespace zcsd {

// ---------------------------------------------------------------------------
// blocked Householder QR (qr.hip)
enum class QRShape { General, Stacked };

struct QRWork {
  int nb = 32, K = 0;
  long long ldv = 0;
  double* V = nullptr;  long long sV = 0;   // K panels of ldv x nb per problem
  double* T = nullptr;  long long sT = 0;   // K blocks of nb x nb per problem
  double* W = nullptr;  double* W2 = nullptr; long long sW = 0;  // nbo x n scratch per problem
  TsqrScratch ts;                                                 // tall-panel scratch
  double* ws = nullptr; size_t ws_elems = 0;                      // split-K workspace
  // two-level blocking (nbo > 0): outer blocks of nbo columns, each made of
  // nbo / nb inner panels; V holds Ko outer blocks of ldv x nbo, To their
  // nbo x nbo compact-WY factors, Tin the inner factors of the current block
  int nbo = 0, Ko = 0;
  double* To = nullptr; long long sTo = 0;
  double* Tin = nullptr; long long sTin = 0;
  double* G = nullptr; long long sG = 0;
  // inner-panel updates (two-level): per-problem partial products and counters
  double* pu_part = nullptr; long long sPart = 0;
  unsigned* pu_cnt = nullptr;
  Arena* ar = nullptr;
};

// qcols > n: room for orgqr_batched to form a Q with qcols columns
QRWork qr_work_alloc(Arena& ar, QRShape shape, int batch, int m, int n, int nb, int qcols = 0);
// arena bytes taken by qr_work_alloc
size_t qr_work_bytes(QRShape shape, int batch, int m, int n, int nb, int qcols = 0);
// In place: M_b (m x n, or 2n x n for Stacked) -> R in its top n x n upper triangle,
// zeros below; reflectors kept in wk.
void geqrf_batched(int batch, QRShape shape, int m, int n, double* M, long long ldm, long long sM,
                   QRWork& wk, hipStream_t s);
// Q_b = H_1 ... H_K [scale_b I_nq; 0] (m x nq, nq = max(n, qcols)); d_scale may be
// NULL (scale 1).  qcols > n (General shape, workspace from qr_work_alloc with
// the same qcols): the n reflectors of an m x n factorization extended to more
// columns, e.g. the whole m x m orthogonal factor (LAPACK's orgqr with k < n).
void orgqr_batched(int batch, QRShape shape, int m, int n, double* Q, long long ldq, long long sQ,
                   const double* d_scale, const QRWork& wk, hipStream_t s, int qcols = 0);

// ---------------------------------------------------------------------------
// element-wise helpers beyond zcsd_internal.h (elem.hip)
// X_b = v_b I (m x n), v_b = d_vals[b] when d_vals != NULL else v
void set_identity_scaled(int batch, int m, int n, const double* d_vals, double v, double* X,
                         long long ldx, long long sx, hipStream_t s);

// ---------------------------------------------------------------------------
// Cholesky with inverse factor (chol.hip): for SPD A_b (n x n, lower/upper both
// read symmetrically from the upper triangle): R_b upper with R^T R = A and
// Ri_b = R^{-1}; both n x n with ld n, stride n*n.  A is overwritten.
void chol_inv_batched(int batch, int n, double* A, long long lda, long long sA, double* R,
                      double* Ri, Arena& ar, hipStream_t s);
// Upper-triangular inverse Ri = R^{-1} (n x n), level-parallel recursion.
void trtri_upper_batched(int batch, int n, const double* R, long long ldr, long long sR, double* Ri,
                         long long ldi, long long sI, Arena& ar, hipStream_t s);

}  // namespace zcsd
