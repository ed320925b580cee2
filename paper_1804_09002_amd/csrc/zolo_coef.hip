// Zolotarev coefficients on the host (Sec. 5, Zolo-pd).
//
// The type (2r+1, 2r) Zolotarev function on [l, 1] is
//     Z(x) = M x prod_{j=1..r} (x^2 + c_{2j}) / (x^2 + c_{2j-1}),
//     c_i = l^2 sn^2(u_i; l') / cn^2(u_i; l'),  u_i = i K(l') / (2r+1),
// with partial fractions prod_j (y + c_{2j})/(y + c_{2j-1}) = 1 + sum_j a_j / (y + c_{2j-1}),
// a_j = -prod_k (c_{2j-1} - c_{2k}) / prod_{k != j} (c_{2j-1} - c_{2k-1}),
// and M fixed by Z(1) = 1.
//
// For l down to 1e-15 the modulus l' = sqrt(1 - l^2) rounds to 1 and the
// textbook AGM evaluation of sn/cn loses all accuracy.  We use instead the
// Jacobi imaginary transformation sc(u; l') = -i sn(iu; l) and the theta
// series of sn for the complementary modulus l, whose nome q = exp(-L),
// L = pi K(l') / K(l), is tiny when l is small:
//     l sc(u_i; l') = 4 S2 N_i / (theta3(0) theta4(i v_i)),
//     S2  = sum_{n>=0} q^{n(n+1)},
//     N_i = sum_{n>=0} (-1)^n q^{1/2 + n(n+1)} sinh((2n+1) v_i),
//     theta4(i v) = 1 + 2 sum_{n>=1} (-1)^n q^{n^2} cosh(2 n v),
//     v_i = (i / (2r+1)) L / 2,
// every term evaluated as an exponential of a non-positive argument (no
// overflow, no cancellation of large terms).  K values come from the
// arithmetic-geometric mean, K(k) = pi / (2 AGM(1, sqrt(1 - k^2))), so
// L = pi AGM(1, l') / AGM(1, l).  Arithmetic is long double (x87, 64-bit
// mantissa) and results are rounded to double once.
#include <cmath>

#include "zcsd_internal.h"
#include "zcsd_zolo.h"

namespace zcsd {

typedef long double ld;

static ld agm(ld a, ld b) {
  for (int it = 0; it < 200; ++it) {
    const ld an = 0.5L * (a + b), bn = sqrtl(a * b);
    a = an;
    b = bn;
    if (fabsl(a - b) <= 1e-19L * a) break;
  }
  return 0.5L * (a + b);
}

// c[0..2r-1] = c_1..c_2r for lower bound l (long double)
static void zolo_c(ld l, int r, ld* c) {
  const ld lp = sqrtl((1.0L - l) * (1.0L + l));
  const ld PI = 3.141592653589793238462643383279502884L;
  const ld L = PI * agm(1.0L, lp) / agm(1.0L, l);
  ld th3 = 1.0L, S2 = 0.0L;
  for (int n = 0; n < 64; ++n) {
    const ld t2 = expl(-L * (ld)n * (ld)(n + 1));
    S2 += t2;
    if (n >= 1) th3 += 2.0L * expl(-L * (ld)n * (ld)n);
    if (t2 < 1e-30L && n >= 1) break;
  }
  for (int i = 1; i <= 2 * r; ++i) {
    const ld v = ((ld)i / (ld)(2 * r + 1)) * 0.5L * L;
    ld num = 0.0L;
    for (int n = 0; n < 64; ++n) {
      const ld e0 = -L * (0.5L + (ld)n * (ld)(n + 1));
      const ld t = 0.5L * (expl(e0 + (2 * n + 1) * v) - expl(e0 - (2 * n + 1) * v));
      num += (n & 1) ? -t : t;
      if (fabsl(t) < 1e-30L * fabsl(num) && n >= 1) break;
    }
    ld th4 = 1.0L;
    for (int n = 1; n < 64; ++n) {
      const ld e0 = -L * (ld)n * (ld)n;
      const ld t = expl(e0 + 2 * n * v) + expl(e0 - 2 * n * v);  // 2 q^{n^2} cosh(2 n v)
      th4 += (n & 1) ? -t : t;
      if (fabsl(t) < 1e-30L) break;
    }
    const ld lsc = 4.0L * S2 * num / (th3 * th4);
    c[i - 1] = lsc * lsc;
  }
}

ZoloStepCoef zolo_step(double ell, int r) {
  if (!(ell > 0.0 && ell <= 1.0) || r < 1 || r > ZOLO_RMAX)
    throw ArgError("zolo_step: need 0 < l <= 1 and 1 <= r <= 8");
  ZoloStepCoef z;
  z.r = r;
  z.ell = ell;
  ld c[2 * ZOLO_RMAX];
  zolo_c((ld)ell, r, c);
  ld a[ZOLO_RMAX];
  for (int j = 0; j < r; ++j) {
    ld num = 1.0L, den = 1.0L;
    for (int k = 0; k < r; ++k) {
      num *= c[2 * j] - c[2 * k + 1];
      if (k != j) den *= c[2 * j] - c[2 * k];
    }
    a[j] = -num / den;
  }
  ld prod = 1.0L;
  for (int j = 0; j < r; ++j) prod *= (1.0L + c[2 * j + 1]) / (1.0L + c[2 * j]);
  const ld M = 1.0L / prod;
  // l_next = Z(l) in the product form
  const ld x = (ld)ell;
  ld zx = M * x;
  for (int j = 0; j < r; ++j) zx *= (x * x + c[2 * j + 1]) / (x * x + c[2 * j]);
  for (int i = 0; i < 2 * r; ++i) z.c[i] = (double)c[i];
  for (int j = 0; j < r; ++j) z.a[j] = (double)a[j];
  z.M = (double)M;
  z.ell_next = (double)(zx < 1.0L ? zx : 1.0L);
  z.one_minus_next = (double)(1.0L - (zx < 1.0L ? zx : 1.0L));
  return z;
}

ZoloPlan zolo_plan(double ell, int r) {
  ZoloPlan p;
  p.step[0] = zolo_step(ell, r);
  p.step[1] = zolo_step(p.step[0].ell_next, r);
  p.resid = p.step[1].one_minus_next;
  return p;
}

int zolo_choose_r(double ell, double tol) {
  for (int r = 1; r <= ZOLO_RMAX; ++r) {
    ZoloPlan p = zolo_plan(ell, r);
    if (p.resid <= tol) return r;
  }
  return 0;
}

}  // namespace zcsd

extern "C" {

zcsd_status zcsd_zolo_coeffs(double ell, int r, double* h_c, double* h_a, double* h_M,
                             double* h_ell_next) {
  if (!(ell > 0.0 && ell <= 1.0) || r < 1 || r > zcsd::ZOLO_RMAX) return ZCSD_EINVAL;
  try {
    zcsd::ZoloStepCoef z = zcsd::zolo_step(ell, r);
    for (int i = 0; i < 2 * r; ++i)
      if (h_c) h_c[i] = z.c[i];
    for (int j = 0; j < r; ++j)
      if (h_a) h_a[j] = z.a[j];
    if (h_M) *h_M = z.M;
    if (h_ell_next) *h_ell_next = z.ell_next;
  } catch (...) {
    return ZCSD_EINVAL;
  }
  return ZCSD_OK;
}

int zcsd_zolo_choose_r(double ell, double tol) {
  if (!(ell > 0.0 && ell <= 1.0)) return 0;
  try {
    return zcsd::zolo_choose_r(ell, tol);
  } catch (...) {
    return 0;
  }
}

}  // extern "C"
