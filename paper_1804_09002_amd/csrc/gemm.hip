// FP64 matrix product on the gfx950 matrix cores (v_mfma_f64_16x16x4f64).
//
// C_b = alpha op(A_b) op(B_b) + beta C_b, column-major, batched with element
// strides.  Every dense contraction of the Zolo-csd path (the trailing updates
// and Q formation of the blocked Householder QR, the Cholesky and triangular
// inverse recursions, the Zolotarev combines, B, U_i = W_i V1, V1^T H_i V1)
// goes through this kernel.
//
// Tiling: a 256-thread workgroup (4 wave64s in a 2 x 2 grid) owns a BM x BN
// tile of C, with registers capped so that two workgroups share a CU (their
// MFMA streams hide each other's LDS and global latency: +35 % over one); each wave owns WM x WN = (BM/2) x (BN/2) and issues
// (WM/16) x (WN/16) MFMA 16x16x4 blocks per k-step of 4.  A and B tiles of
// depth BK are staged through LDS (k-major), with the next tile's global loads
// issued into registers before the current tile's MFMAs.
//
// Lane layout of v_mfma_f64_16x16x4f64 (wave64): input a[i][k] comes from
// lane i + 16k, input b[k][j] from lane j + 16k, and output d[i][j] is item
// i / 4 of lane j + 16 (i % 4).  The kernel feeds op(B)^T as the MFMA "a"
// operand and op(A)^T as "b", so the accumulator holds C^T: lane l, item v is
// C[row0 + l % 16][col0 + l / 16 + 4 v], and 16 consecutive lanes store 16
// consecutive rows of one column of C (a 128-byte coalesced segment).
//
// The same kernel also runs the products of the mixed-precision mode on the
// FP32 matrix cores (F32 = true): operands are rounded to FP32 as they are
// staged into LDS, accumulation is FP32 (v_mfma_f32_16x16x4f32, twice the
// FP64 rate), results are written in FP64.  FP32 tiles are 32 deep, so LDS
// holds the same bytes as the 16-deep FP64 tiles.  Lane layout of the FP32
// instruction: output d[i][j] is item i % 4 of lane j + 16 (i / 4), so lane
// l, item v holds C[row0 + l % 16][col0 + 4 (l / 16) + v].
#include <algorithm>
#include <array>
#include <cstdlib>
#include <string>

#include <hip/hip_ext.h>

#include "zcsd_internal.h"
#include "zcsd_prof.h"

namespace zcsd {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// precision scope of the products (GemmLowpScope / GemmFp64Scope) and the
// count of FP32 product launches, per host thread
namespace {
thread_local int g_lowp_mode = 0;  // 0 FP64, 1 FP32 where it pays, 2 FP32 always
// products with at least this many 128 x 128 output tiles (over the batch)
// take the 128 x 128 tiling, the others the 64 x 64 one (GemmTileScope)
thread_local int g_tile128_min = kGemmTile128MinDefault;
thread_local long long g_lowp_launches = 0;
}

// arithmetic of the two instantiations: LDS element type, accumulator, MFMA
// step, and the column offset of accumulator item v in lane group lk
template <bool F32>
struct Mma;
template <>
struct Mma<false> {
  using T = double;
  using Acc = d4;
  static __device__ __forceinline__ Acc step(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int col(int lk, int v) { return lk + 4 * v; }
};
template <>
struct Mma<true> {
  using T = float;
  using Acc = f4;
  static __device__ __forceinline__ Acc step(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int col(int lk, int v) { return 4 * lk + v; }
};

template <int BM, int BN, int BK, bool TA, bool TB, bool F32>
__global__ __launch_bounds__(256, 2) void dgemm_kernel(
    int m, int n, int k, const double* __restrict__ A, long long lda, long long sA,
    const double* __restrict__ B, long long ldb, long long sB, double* __restrict__ C,
    long long ldc, long long sC, double alpha, double beta, int nb1, long long sA2, long long sB2,
    long long sC2, int nprob, int kchunk, double* ws, int sym_upper, int tri, int kseg,
    int order) {
  // tile (bx, by) of problem zp; order 0: the grid's (x, y) and z = (split,
  // problem); order 1, 2 (square products whose operands make k >= max(i, j)
  // the only nonzero range, so a tile's work falls with max(x, y)): a linear
  // grid over (tile, problem) with the problem fastest and the heaviest tiles
  // first, so that no long tile starts at the end of the launch.  Order 1
  // walks shells of max(x, y) = m (tiles (0..m, m) then (m, 0..m-1)); order 2
  // (symmetric products) the upper tiles x <= y column by column.
  int bx, by, zp, split;
  if (order == 0) {
    if (sym_upper && blockIdx.x > blockIdx.y) return;  // tile below the diagonal (BM == BN)
    bx = blockIdx.x;
    by = blockIdx.y;
    zp = blockIdx.z % nprob;
    split = blockIdx.z / nprob;
  } else {
    const long long L = blockIdx.x;
    zp = (int)(L % nprob);
    split = 0;
    const long long t = L / nprob;
    if (order == 1) {
      int m = (int)sqrt((double)t);
      while ((long long)m * m > t) --m;
      while ((long long)(m + 1) * (m + 1) <= t) ++m;
      const int r = (int)(t - (long long)m * m);
      if (r <= m) {
        bx = r;
        by = m;
      } else {
        bx = m;
        by = r - m - 1;
      }
    } else {
      int y = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
      while ((long long)y * (y + 1) / 2 > t) --y;
      while ((long long)(y + 1) * (y + 2) / 2 <= t) ++y;
      by = y;
      bx = (int)(t - (long long)y * (y + 1) / 2);
    }
  }
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int NA = BM * BK / 256, NB = BN * BK / 256;
  static_assert(NA * 256 == BM * BK && NB * 256 == BN * BK, "tile/threads mismatch");
  using M = Mma<F32>;
  using T = typename M::T;
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int i0 = bx * BM;
  const int j0 = by * BN;
  const long long b1 = zp % nb1, b2 = zp / nb1;  // problem index (b1, b2)
  A += b1 * sA + b2 * sA2;
  B += b1 * sB + b2 * sB2;
  C += b1 * sC + b2 * sC2;
  if (kchunk > 0) {
    // this workgroup owns k in [split*kchunk, min(k, (split+1)*kchunk)) and writes
    // its partial product (alpha = 1, beta = 0) to the workspace slab (ld m)
    const int kb = split * kchunk;
    A += TA ? (long long)kb : (long long)kb * lda;
    B += TB ? (long long)kb * ldb : (long long)kb;
    k = min(kchunk, k - kb);
    C = ws + ((long long)split * nprob + zp) * (long long)m * n;
    ldc = m;
    alpha = 1.0;
    beta = 0.0;
  }

  T ra[NA], rb[NB];
  // with the large tiles, a tile wholly inside C (and a k-tile wholly inside
  // k) loads and stores without per-element bounds checks (measured faster
  // for 128 x 128 tiles, slower for the small split-K products of 64 x 64)
  const bool full_mn = (BM >= 128) && (i0 + BM <= m) && (j0 + BN <= n);
  auto load_tiles = [&](int k0, int kl) {
    if (full_mn && k0 + BK <= kl) {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int e = tid + 256 * q;
        int i, kk;
        if (!TA) { i = e % BM; kk = e / BM; } else { kk = e % BK; i = e / BK; }
        const int gi = i0 + i, gk = k0 + kk;
        ra[q] = (T)(TA ? A[gk + (long long)gi * lda] : A[gi + (long long)gk * lda]);
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int e = tid + 256 * q;
        int j, kk;
        if (!TB) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
        const int gj = j0 + j, gk = k0 + kk;
        rb[q] = (T)(TB ? B[gj + (long long)gk * ldb] : B[gk + (long long)gj * ldb]);
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      int i, kk;
      if (!TA) { i = e % BM; kk = e / BM; } else { kk = e % BK; i = e / BK; }
      const int gi = i0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < m && gk < kl) v = TA ? A[gk + (long long)gi * lda] : A[gi + (long long)gk * lda];
      ra[q] = (T)v;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      int j, kk;
      if (!TB) { kk = e % BK; j = e / BK; } else { j = e % BN; kk = e / BN; }
      const int gj = j0 + j, gk = k0 + kk;
      double v = 0.0;
      if (gj < n && gk < kl) v = TB ? B[gj + (long long)gk * ldb] : B[gk + (long long)gj * ldb];
      rb[q] = (T)v;
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

  typename M::Acc acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) acc[x][y] = typename M::Acc{0, 0, 0, 0};

  const int lr = lane & 15;   // row (of the 16-block) this lane feeds / owns
  const int lk = lane >> 4;   // k index within the k-step of 4

  // k-range of this tile: K is a sequence of segments of length seg; within a
  // segment, products that the triangular structure of op(A) or op(B) makes
  // zero are skipped (tri bits: 1 op(A) upper, k >= i; 2 op(A) lower, k <= i;
  // 4 op(B) upper, k <= j; 8 op(B) lower, k >= j)
  int seg = k, nseg = 1, klo = 0, khi = k;
  if (tri && kchunk == 0 && kseg > 0) {
    seg = kseg;
    nseg = k / kseg;
    khi = seg;
    if (tri & 1) klo = max(klo, i0);
    if (tri & 8) klo = max(klo, j0);
    if (tri & 2) khi = min(khi, i0 + BM);
    if (tri & 4) khi = min(khi, j0 + BN);
    klo = (klo / BK) * BK;
  }
  const int nkt = (khi > klo) ? (khi - klo + BK - 1) / BK : 0;
  const int total = nseg * nkt;
  auto kstart = [&](int t) { return (t / nkt) * seg + klo + (t % nkt) * BK; };
  auto klim = [&](int t) { return (t / nkt) * seg + khi; };

  if (total > 0) load_tiles(kstart(0), klim(0));
  for (int t = 0; t < total; ++t) {
    __syncthreads();
    store_tiles();
    __syncthreads();
    if (t + 1 < total) load_tiles(kstart(t + 1), klim(t + 1));
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T fa[TM], fb[TN];
#pragma unroll
      for (int x = 0; x < TM; ++x) fa[x] = As[kk + lk][wm * WM + x * 16 + lr];
#pragma unroll
      for (int y = 0; y < TN; ++y) fb[y] = Bs[kk + lk][wn * WN + y * 16 + lr];
#pragma unroll
      for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y) acc[x][y] = M::step(fb[y], fa[x], acc[x][y]);
    }
  }

  // epilogue: lane owns C[row][col + 4v].  With beta != 0 the old values of a
  // row tile are all loaded, then the results formed, then stored: loads
  // interleaved with stores of the same array would each wait for the store
  // before them (one memory round trip per element)
  const bool rd = beta != 0.0;
  if (full_mn) {
#pragma unroll
    for (int x = 0; x < TM; ++x) {
      const int row = i0 + wm * WM + x * 16 + lr;
      double o[TN][4];
      if (rd) {
#pragma unroll
        for (int y = 0; y < TN; ++y)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            o[y][v] = C[row + (long long)(j0 + wn * WN + y * 16 + M::col(lk, v)) * ldc];
#pragma unroll
        for (int y = 0; y < TN; ++y)
#pragma unroll
          for (int v = 0; v < 4; ++v) o[y][v] = alpha * (double)acc[x][y][v] + beta * o[y][v];
      } else {
#pragma unroll
        for (int y = 0; y < TN; ++y)
#pragma unroll
          for (int v = 0; v < 4; ++v) o[y][v] = alpha * (double)acc[x][y][v];
      }
#pragma unroll
      for (int y = 0; y < TN; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) C[row + (long long)(j0 + wn * WN + y * 16 + M::col(lk, v)) * ldc] = o[y][v];
    }
    return;
  }
#pragma unroll
  for (int x = 0; x < TM; ++x) {
    const int row = i0 + wm * WM + x * 16 + lr;
    if (row >= m) continue;
    double o[TN][4];
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = j0 + wn * WN + y * 16 + M::col(lk, v);
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
        const int col = j0 + wn * WN + y * 16 + M::col(lk, v);
        if (col < n) C[row + (long long)col * ldc] = o[y][v];
      }
  }
}

// C_p = alpha sum_s ws[s][p] + beta C_p  (split-K reduction, deterministic order)
__global__ void splitk_reduce_kernel(int m, int n, int nprob, int nsplit, const double* __restrict__ ws,
                                     double* C, long long ldc, long long sC, int nb1,
                                     long long sC2, double alpha, double beta) {
  const int zp = blockIdx.y;
  const long long b1 = zp % nb1, b2 = zp / nb1;
  double* Cp = C + b1 * sC + b2 * sC2;
  const long long mn = (long long)m * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < mn;
       e += (long long)gridDim.x * blockDim.x) {
    // the partials (at most 16) and the old value loaded together, then summed in order
    const int i = (int)(e % m), j = (int)(e / m);
    double* c = Cp + i + (long long)j * ldc;
    double pv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) pv[q] = (q < nsplit) ? ws[((long long)q * nprob + zp) * mn + e] : 0.0;
    const double old = (beta == 0.0) ? 0.0 : *c;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (q < nsplit) s += pv[q];
    *c = (beta == 0.0) ? alpha * s : alpha * s + beta * old;
  }
}

template <int BM, int BN, int BK, bool F32>
static const char* tile_name(int ta, int tb) {
  // initialised once (thread-safe), read by every launch
  static const std::array<std::string, 4> names = [] {
    std::array<std::string, 4> a;
    for (int i = 0; i < 4; ++i)
      a[i] = std::string(F32 ? "gemm_f32acc_" : "dgemm_") + std::to_string(BM) + "x" +
             std::to_string(BN) + "_" + ((i & 2) ? "T" : "N") + ((i & 1) ? "T" : "N");
    return a;
  }();
  return names[(ta ? 2 : 0) + (tb ? 1 : 0)].c_str();
}

// Flops of the tiles a launch computes: tiles below the diagonal of a
// symmetric product are skipped, and so are the k ranges that triangular
// operands make zero (the same ranges the kernel skips).  Evaluated only while
// the profiler records.
template <int BM, int BN, int BK>
static double computed_flops(const GemmBatch& g, bool split) {
  const double nprob = (double)g.batch * g.batch2;
  const bool upper = g.sym_upper || g.upper_only;
  if (!upper && (!g.tri || split)) return 2.0 * g.m * (double)g.n * g.k * nprob;
  const int gx = (g.m + BM - 1) / BM, gy = (g.n + BN - 1) / BN;
  double f = 0.0;
  for (int by = 0; by < gy; ++by)
    for (int bx = 0; bx < gx; ++bx) {
      if (upper && bx > by) continue;
      const int i0 = bx * BM, j0 = by * BN;
      double kr = g.k;
      if (g.tri && !split && g.kseg > 0) {
        int klo = 0, khi = g.kseg;
        if (g.tri & 1) klo = std::max(klo, i0);
        if (g.tri & 8) klo = std::max(klo, j0);
        if (g.tri & 2) khi = std::min(khi, i0 + BM);
        if (g.tri & 4) khi = std::min(khi, j0 + BN);
        klo = (klo / BK) * BK;
        kr = (double)(g.k / g.kseg) * std::max(0, khi - klo);
      }
      f += 2.0 * std::min(BM, g.m - i0) * (double)std::min(BN, g.n - j0) * kr;
    }
  return f * nprob;
}

template <int BM, int BN, int BK, bool F32>
static void launch_tile(const GemmBatch& g, hipStream_t s, int ksplit) {
  const double nprob_d = (double)g.batch * g.batch2;
  // the events of the profiler are attached to the product's dispatches (the
  // first chunk's start, the last chunk's end; a split-K reduction is not
  // included): about 1500 launches a CSD, whose marker packets would
  // lengthen the profiled run by several ms
  ProfScope prof(tile_name<BM, BN, BK, F32>(g.transA, g.transB), s,
                 prof_on() ? computed_flops<BM, BN, BK>(g, ksplit > 1) : 0.0,
                 8.0 * nprob_d * ((double)g.m * g.k + (double)g.k * g.n + (g.beta != 0.0 ? 2.0 : 1.0) * g.m * g.n),
                 /*ext=*/true);
  const int gx = (g.m + BM - 1) / BM, gy = (g.n + BN - 1) / BN;
  if (g.batch > 65535) throw ArgError("dgemm: batch too large");
  int kchunk = 0;
  if (ksplit > 1) {
    kchunk = (g.k + ksplit - 1) / ksplit;
    kchunk = ((kchunk + BK - 1) / BK) * BK;
    ksplit = (g.k + kchunk - 1) / kchunk;
  }
  const int nsplit = std::max(1, ksplit);
  if (nsplit > 16) throw ArgError("dgemm: at most 16 k-splits");
  // the z dimension enumerates (split, b2, b1); chunk over b2 to stay within 65535
  const int per = std::max(1, 65535 / std::max(1, g.batch * nsplit));
  if (kchunk > 0 && per < g.batch2) throw ArgError("dgemm: split-K batch too large");
  for (int c0 = 0; c0 < g.batch2; c0 += per) {
    const int nc = std::min(per, g.batch2 - c0);
    const int nprob = g.batch * nc;
    // heavy tiles first for square products with k >= max(i, j), and only the
    // upper tiles of symmetric products (see the kernel).  Measured: with the
    // grid's own order neither skipping the lower tiles of a symmetric
    // product nor the light tiles of a triangular one shortened the launch
    // (8 symmetric 4096^2 products took 17.8 ms against 18.0 ms for the full
    // ones), since a launch lasts as long as the most loaded CU
    int order = 0;
    if (kchunk == 0 && gx == gy && !g.upper_only) {
      if (g.sym_upper && (g.tri == 0 || (g.tri & 9) == 9)) order = 2;
      else if (!g.sym_upper && (g.tri & 9) == 9) order = 1;
    }
    const long long lin = (order == 2 ? (long long)gx * (gx + 1) / 2 : (long long)gx * gy) * nprob;
    dim3 grid = order ? dim3((unsigned)lin, 1, 1) : dim3(gx, gy, nprob * nsplit);
    dim3 block(256);
    const double* A = g.A + (long long)c0 * g.sA2;
    const double* B = g.B + (long long)c0 * g.sB2;
    double* C = g.C + (long long)c0 * g.sC2;
    hipEvent_t ev0 = (c0 == 0) ? prof.ext_start() : nullptr;
    hipEvent_t ev1 = (c0 + per >= g.batch2) ? prof.ext_stop() : nullptr;
#define ZCSD_GEMM_LAUNCH(TA_, TB_)                                                        \
  hipExtLaunchKernelGGL((dgemm_kernel<BM, BN, BK, TA_, TB_, F32>), grid, block, 0, s, ev0, ev1, 0, g.m, g.n, g.k, A, \
                     g.lda, g.sA, B, g.ldb, g.sB, C, g.ldc, g.sC, g.alpha, g.beta, g.batch,     \
                     g.sA2, g.sB2, g.sC2, nprob, kchunk, g.ws, (g.sym_upper || g.upper_only) ? 1 : 0, g.tri, \
                     g.kseg, order)
    if (!g.transA && !g.transB) ZCSD_GEMM_LAUNCH(false, false);
    else if (!g.transA && g.transB) ZCSD_GEMM_LAUNCH(false, true);
    else if (g.transA && !g.transB) ZCSD_GEMM_LAUNCH(true, false);
    else ZCSD_GEMM_LAUNCH(true, true);
#undef ZCSD_GEMM_LAUNCH
    ZCSD_CHECK_LAUNCH();
    if (kchunk > 0) {
      const long long mn = (long long)g.m * g.n;
      const unsigned gxr = (unsigned)std::max<long long>(1, std::min<long long>((mn + 255) / 256, 1024));
      hipLaunchKernelGGL(splitk_reduce_kernel, dim3(gxr, nprob), dim3(256), 0, s, g.m, g.n, nprob,
                         nsplit, g.ws, C, g.ldc, g.sC, g.batch, g.sC2, g.alpha, g.beta);
      ZCSD_CHECK_LAUNCH();
    }
  }
}

void dgemm(const GemmBatch& g, hipStream_t s) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0 || g.batch2 <= 0) return;
  if (g.sym_upper && (g.m != g.n || g.beta != 0.0))
    throw ArgError("dgemm: a symmetric product needs m == n and beta == 0");
  if (g.upper_only && g.m != g.n) throw ArgError("dgemm: an upper-triangle product needs m == n");
  if (g.tri && (g.kseg <= 0 || g.k % g.kseg != 0))
    throw ArgError("dgemm: triangular operands need k to be a multiple of kseg");
  if (g.k <= 0) {
    // C = beta C
    if (g.beta != 1.0)
      for (int c = 0; c < g.batch2; ++c)
        copy_scale(g.batch, g.m, g.n, g.beta, g.C + c * g.sC2, g.ldc, g.sC, g.C + c * g.sC2, g.ldc,
                   g.sC, s);
    return;
  }
  const long long nprob = (long long)g.batch * g.batch2;
  const long long tiles128 = (long long)((g.m + 127) / 128) * ((g.n + 127) / 128) * nprob;
  // inside a GemmLowpScope the FP32 matrix cores take the products where they
  // did not measure slower than FP64: dense products with op(B) = B (4096^3
  // NN: 90 against 60 TFLOP/s); transposed-B products (2 x 4096 x 4096 x
  // 16384 NT: 52 against 61) and triangular ones (equal or slower) stay FP64
  const int lm = g_lowp_mode;
  const bool f32 = lm == 2 || (lm == 1 && !g.tri && !g.transB);
  if (f32) ++g_lowp_launches;
  if (tiles128 >= g_tile128_min) {
    if (f32) launch_tile<128, 128, 32, true>(g, s, 1);
    else launch_tile<128, 128, 16, false>(g, s, 1);
    return;
  }
  // few output tiles and a long k: split k across workgroups when a workspace is given
  const long long tiles64 = (long long)((g.m + 63) / 64) * ((g.n + 63) / 64) * nprob;
  int ksplit = 1;
  static const bool no_split = [] {
    const char* e = std::getenv("ZCSD_NO_SPLITK");
    return e && e[0] == '1';
  }();
  if (g.ws && !no_split && !g.upper_only && tiles64 < 256 && g.k >= 1024) {
    ksplit = (int)std::min<long long>(std::min<long long>(g.k / 256, 16),
                                      std::max<long long>(2, 512 / std::max<long long>(1, tiles64)));
    while (ksplit > 1 && (size_t)ksplit * nprob * g.m * g.n > g.ws_elems) --ksplit;
  }
  if (f32) launch_tile<64, 64, 32, true>(g, s, ksplit);
  else launch_tile<64, 64, 16, false>(g, s, ksplit);
}

// ---------------------------------------------------------------------------
// precision scopes of the mixed mode (see zcsd_internal.h)
long long gemm_lowp_launches() { return g_lowp_launches; }
GemmLowpScope::GemmLowpScope(bool on, bool always) : on_(on), saved_(g_lowp_mode) {
  if (on_) g_lowp_mode = always ? 2 : 1;
}
GemmLowpScope::~GemmLowpScope() {
  if (on_) g_lowp_mode = saved_;
}
GemmFp64Scope::GemmFp64Scope(bool on) : on_(on), saved_(g_lowp_mode) {
  if (on_) g_lowp_mode = 0;
}
GemmFp64Scope::~GemmFp64Scope() {
  if (on_) g_lowp_mode = saved_;
}
bool gemm_lowp_active() { return g_lowp_mode > 0; }
GemmTileScope::GemmTileScope(int min_tiles) : saved_(g_tile128_min) {
  if (min_tiles > 0) g_tile128_min = min_tiles;
}
GemmTileScope::~GemmTileScope() { g_tile128_min = saved_; }

}  // namespace zcsd
