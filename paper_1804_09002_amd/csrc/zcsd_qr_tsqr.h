// TSQR panel factorisation with Householder reconstruction (qr_tsqr.hip).
#pragma once
#include "zcsd_internal.h"

namespace zcsd {

constexpr int TS_MB = 256;    // rows per block of the first level
constexpr int TS_PMAX = 17;   // at most this many blocks (the tree QR holds P*32 rows)

struct TsqrScratch {
  double* Rstack = nullptr;  // (P w) x w stacked R factors, ld P*32
  double* Qtop = nullptr;    // (P w) x w: Householder vectors Y_top of the tree QR
  double* Z = nullptr;       // 32 x 32: T_top Y_top(0:w, :)^T
  double* Tloc = nullptr;    // P blocks of 32 x 32
  double* U = nullptr;       // 32 x 32
  double* L = nullptr;       // 32 x 32
  double* S = nullptr;       // 32
  long long stride = 0;      // per problem
};

bool tsqr_panel_fits(int h, int w);
TsqrScratch tsqr_scratch_alloc(Arena& ar, int batch);
size_t tsqr_scratch_bytes(int batch);  // arena bytes of tsqr_scratch_alloc
// Same contract as the one-workgroup panel: reads the panel's rows (two
// segments) of M, writes R into the top w logical rows and zeros below,
// V (h x w, unit lower trapezoidal, ld ldv) and T (32 x 32, upper).  Logical
// rows of the second segment go to rows vr2.. of V (vr2 < 0: right after the
// first segment).
void tsqr_panel(int batch, double* M, long long ldm, long long sM, int c0, int w, int r1a, int r1b,
                int r2a, int r2b, double* V, long long ldv, long long sV, int vr2, double* T,
                long long sT, const TsqrScratch& sc, hipStream_t s);

}  // namespace zcsd
