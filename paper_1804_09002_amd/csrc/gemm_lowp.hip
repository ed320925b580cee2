// Matrix product on the FP32 matrix cores (v_mfma_f32_16x16x4f32) for FP64
// operands: C = alpha op(A) op(B) + beta C with A, B rounded to FP32 as they
// are staged into LDS, FP32 accumulation, and the FP64 epilogue.  Used by the
// mixed-precision mode for the products whose error a later FP64 refinement
// removes (GemmLowpScope); the tiling follows the FP64 kernel.
//
// Lane layout of v_mfma_f32_16x16x4f32 (wave64): input a[i][k] from lane
// i + 16k, input b[k][j] from lane j + 16k, output d[i][j] is item i % 4 of
// lane j + 16 (i / 4).  Fed with op(B)^T as "a" and op(A)^T as "b", lane l
// item v holds C[row0 + l % 16][col0 + 4 (l / 16) + v].
#include <algorithm>
#include <string>

#include "zcsd_internal.h"
#include "zcsd_prof.h"

namespace zcsd {

typedef float f4 __attribute__((ext_vector_type(4)));

namespace {
thread_local int g_lowp_depth = 0;
}

GemmLowpScope::GemmLowpScope(bool on) : on_(on) {
  if (on_) ++g_lowp_depth;
}
GemmLowpScope::~GemmLowpScope() {
  if (on_) --g_lowp_depth;
}
GemmFp64Scope::GemmFp64Scope() : saved_(g_lowp_depth) { g_lowp_depth = 0; }
GemmFp64Scope::~GemmFp64Scope() { g_lowp_depth = saved_; }
bool gemm_lowp_active() { return g_lowp_depth > 0; }

template <int BM, int BN, int BK, bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void gemm_f32acc_kernel(
    int m, int n, int k, const double* __restrict__ A, long long lda, long long sA,
    const double* __restrict__ B, long long ldb, long long sB, double* __restrict__ C,
    long long ldc, long long sC, double alpha, double beta, int nb1, long long sA2, long long sB2,
    long long sC2, int sym_upper) {
  if (sym_upper && blockIdx.x > blockIdx.y) return;  // tile below the diagonal (BM == BN)
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int NA = BM * BK / 256, NB = BN * BK / 256;
  static_assert(NA * 256 == BM * BK && NB * 256 == BN * BK, "tile/threads mismatch");
  __shared__ float As[BK][BM + 1];
  __shared__ float Bs[BK][BN + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int i0 = blockIdx.x * BM;
  const int j0 = blockIdx.y * BN;
  const long long zp = blockIdx.z;
  const long long b1 = zp % nb1, b2 = zp / nb1;
  A += b1 * sA + b2 * sA2;
  B += b1 * sB + b2 * sB2;
  C += b1 * sC + b2 * sC2;

  float ra[NA], rb[NB];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      int i, kk;
      if (!TA) { i = e % BM; kk = e / BM; } else { kk = e % BK; i = e / BK; }
      const int gi = i0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < m && gk < k) v = TA ? A[gk + (long long)gi * lda] : A[gi + (long long)gk * lda];
      ra[q] = (float)v;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      int j, kk;
      if (!TB) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
      const int gj = j0 + j, gk = k0 + kk;
      double v = 0.0;
      if (gj < n && gk < k) v = TB ? B[gj + (long long)gk * ldb] : B[gk + (long long)gj * ldb];
      rb[q] = (float)v;
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      int i, kk;
      if (!TA) { i = e % BM; kk = e / BM; } else { kk = e % BK; i = e / BK; }
      As[kk][i] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      int j, kk;
      if (!TB) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
      Bs[kk][j] = rb[q];
    }
  };

  f4 acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) acc[x][y] = f4{0.f, 0.f, 0.f, 0.f};

  const int lr = lane & 15;
  const int lk = lane >> 4;

  if (k > 0) load_tiles(0);
  for (int k0 = 0; k0 < k; k0 += BK) {
    __syncthreads();
    store_tiles();
    __syncthreads();
    if (k0 + BK < k) load_tiles(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      float fa[TM], fb[TN];
#pragma unroll
      for (int x = 0; x < TM; ++x) fa[x] = As[kk + lk][wm * WM + x * 16 + lr];
#pragma unroll
      for (int y = 0; y < TN; ++y) fb[y] = Bs[kk + lk][wn * WN + y * 16 + lr];
#pragma unroll
      for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(fb[y], fa[x], acc[x][y], 0, 0, 0);
    }
  }

  // a row tile's old values loaded together, then the results, then the
  // stores (loads interleaved with stores of C would each wait for the last store)
  const bool rd = beta != 0.0;
#pragma unroll
  for (int x = 0; x < TM; ++x) {
    const int row = i0 + wm * WM + x * 16 + lr;
    if (row >= m) continue;
    double o[TN][4];
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = j0 + wn * WN + y * 16 + 4 * lk + v;
        o[y][v] = (rd && col < n) ? C[row + (long long)col * ldc] : 0.0;
      }
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double r = alpha * (double)acc[x][y][v];
        o[y][v] = rd ? r + beta * o[y][v] : r;
      }
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = j0 + wn * WN + y * 16 + 4 * lk + v;
        if (col < n) C[row + (long long)col * ldc] = o[y][v];
      }
  }
}

namespace {

template <int BM, int BN, int BK>
const char* lowp_name(int ta, int tb) {
  static std::string store[4];
  const int i = (ta ? 2 : 0) + (tb ? 1 : 0);
  if (store[i].empty())
    store[i] = "gemm_f32acc_" + std::to_string(BM) + "x" + std::to_string(BN) + "_" +
               (ta ? "T" : "N") + (tb ? "T" : "N");
  return store[i].c_str();
}

template <int BM, int BN, int BK>
void launch_lowp(const GemmBatch& g, hipStream_t s) {
  const double nprob_d = (double)g.batch * g.batch2;
  ProfScope prof(lowp_name<BM, BN, BK>(g.transA, g.transB), s,
                 2.0 * g.m * (double)g.n * g.k * nprob_d,
                 8.0 * nprob_d *
                     ((double)g.m * g.k + (double)g.k * g.n + (g.beta != 0.0 ? 2.0 : 1.0) * g.m * g.n));
  const int gx = (g.m + BM - 1) / BM, gy = (g.n + BN - 1) / BN;
  if (g.batch > 65535) throw ArgError("gemm_lowp: batch too large");
  const int per = std::max(1, 65535 / g.batch);
  for (int c0 = 0; c0 < g.batch2; c0 += per) {
    const int nc = std::min(per, g.batch2 - c0);
    dim3 grid(gx, gy, g.batch * nc), block(256);
    const double* A = g.A + (long long)c0 * g.sA2;
    const double* B = g.B + (long long)c0 * g.sB2;
    double* C = g.C + (long long)c0 * g.sC2;
#define ZCSD_LOWP_LAUNCH(TA_, TB_)                                                               \
  hipLaunchKernelGGL((gemm_f32acc_kernel<BM, BN, BK, TA_, TB_>), grid, block, 0, s, g.m, g.n, g.k, \
                     A, g.lda, g.sA, B, g.ldb, g.sB, C, g.ldc, g.sC, g.alpha, g.beta, g.batch,      \
                     g.sA2, g.sB2, g.sC2, (g.sym_upper || g.upper_only) ? 1 : 0)
    if (!g.transA && !g.transB) ZCSD_LOWP_LAUNCH(false, false);
    else if (!g.transA && g.transB) ZCSD_LOWP_LAUNCH(false, true);
    else if (g.transA && !g.transB) ZCSD_LOWP_LAUNCH(true, false);
    else ZCSD_LOWP_LAUNCH(true, true);
#undef ZCSD_LOWP_LAUNCH
    ZCSD_CHECK_LAUNCH();
  }
}

}  // namespace

void gemm_lowp(const GemmBatch& g, hipStream_t s) {
  const long long nprob = (long long)g.batch * g.batch2;
  const long long tiles128 = (long long)((g.m + 127) / 128) * ((g.n + 127) / 128) * nprob;
  if (tiles128 >= 256) launch_lowp<128, 128, 16>(g, s);
  else launch_lowp<64, 64, 16>(g, s);
}

}  // namespace zcsd
