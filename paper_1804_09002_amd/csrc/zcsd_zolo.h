// Zolotarev coefficients and the Zolo-pd / Zolo-eig drivers (internal).
#pragma once
#include "zcsd_internal.h"

namespace zcsd {

constexpr int ZOLO_RMAX = 8;

struct ZoloStepCoef {
  int r = 0;
  double ell = 0.0;               // lower bound of the interval [l, 1]
  double c[2 * ZOLO_RMAX] = {};   // c_1 .. c_2r
  double a[ZOLO_RMAX] = {};       // partial-fraction weights
  double M = 1.0;                 // Z(1) = 1
  double ell_next = 0.0;          // Z(l)
  double one_minus_next = 1.0;    // 1 - Z(l), evaluated before rounding to double
};

struct ZoloPlan {
  ZoloStepCoef step[2];
  double resid = 1.0;             // 1 - l_2
};

ZoloStepCoef zolo_step(double ell, int r);
ZoloPlan zolo_plan(double ell, int r);
int zolo_choose_r(double ell, double tol);

// Batched Zolo-pd on device (zolo_pd.hip).
struct ZoloPdArgs {
  int batch = 1, n = 0;
  double alpha = 1.0;           // X is divided by alpha (alpha >= sigma_max)
  const double* X = nullptr;    // inputs, ld ldx, stride sx
  long long ldx = 0, sx = 0;
  double* W = nullptr;          // outputs (ld n, stride n*n)
  double* H = nullptr;          // may be NULL
  double* X1 = nullptr;         // may be NULL: first iterate
  double eps = 1e-15, tol = 0x1p-53;
  int r_override = 0;
  double ell_override = 0.0;
  bool symmetric_input = false; // X_b symmetric: H not needed, W symmetric
  // mixed mode: the products of iteration 2 (Cholesky form) on the FP32 matrix
  // cores, then one FP64 Newton-Schulz step on the iterate before W and H
  bool lowp_iter2 = false;
  int nb_qr = 32;
};
struct ZoloPdResult {
  int r = 0;
  double ell = 0.0;
  double resid = 1.0;
  int n_qr_terms = 0;
};
ZoloPdResult zolo_pd_batched(const ZoloPdArgs& a, Arena& ar, hipStream_t s);

}  // namespace zcsd
