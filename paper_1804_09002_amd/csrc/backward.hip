// Backward of the CS decomposition: gradients of
//     L = sum_i g_i theta_i + <G1, W1> + <G2, W2>
// with respect to A1 and A2, from the decomposition A1 = U1 C V1^T,
// A2 = U2 S V1^T (C = diag(cos theta), S = diag(sin theta)) and the polar
// factors W_i = U_i V1^T.
//
// * Angles (first-order perturbation of c_i = v_i^T H1 v_i, s_i = v_i^T H2 v_i,
//   Algorithm 1, and theta = atan2(s, c)): d theta_i = -s_i u1_i^T dA1 v_i +
//   c_i u2_i^T dA2 v_i.
// * Polar factor of A = U Sigma V^T: with E = U^T dA V,
//   dW = U [(E - E^T) / (sigma_j + sigma_k)] V^T, hence
//   grad_A <G, W> = U [(M - M^T) / (sigma_j + sigma_k)] V^T, M = U^T G V.
// Both terms share the sandwich U_i (.) V1^T, so per block
//     gA1 = U1 K1 V1^T,  K1 = antisym(M1) / (c_j + c_k) - diag(g s),
//     gA2 = U2 K2 V1^T,  K2 = antisym(M2) / (s_j + s_k) + diag(g c),
// four batched GEMMs per block (G V1, U^T (.), U (.), (.) V1^T) and one
// element-wise kernel.  Pairs with sigma_j + sigma_k = 0 (two zero singular
// values, where W is not differentiable) contribute zero.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "zcsd_api_guard.h"
#include "zcsd_internal.h"

namespace zcsd {

// K_b <- antisym(M_b) / (sigma_j + sigma_k) off the diagonal, dg_j on it, in
// place; sigma_j = cos(theta_j) (blk 0) or sin(theta_j) (blk 1); dg_j =
// -g_j sin(theta_j) (blk 0) or g_j cos(theta_j) (blk 1).  M may be NULL-like
// (has_m == 0): then K is the diagonal alone.  One thread per pair j <= k.
__global__ void csd_bwd_core_kernel(int n, double* K, long long sK, const double* __restrict__ theta,
                                    long long sT, const double* __restrict__ g, int has_m, int blk) {
  const long long b = blockIdx.y;
  double* Kb = K + b * sK;
  const double* th = theta + b * sT;
  const double* gb = g ? g + b * sT : nullptr;
  const long long npairs = (long long)n * (n + 1) / 2;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < npairs;
       e += (long long)gridDim.x * blockDim.x) {
    // e -> (j, k), j <= k, column-major over the upper triangle
    int k = (int)((std::sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
    while ((long long)k * (k + 1) / 2 > e) --k;
    while ((long long)(k + 1) * (k + 2) / 2 <= e) ++k;
    const int j = (int)(e - (long long)k * (k + 1) / 2);
    if (j == k) {
      const double c = cos(th[j]), s = sin(th[j]);
      const double gj = gb ? gb[j] : 0.0;
      Kb[j + (long long)j * n] = (blk == 0) ? -gj * s : gj * c;
    } else {
      double v = 0.0;
      if (has_m) {
        const double sj = (blk == 0) ? cos(th[j]) : sin(th[j]);
        const double sk = (blk == 0) ? cos(th[k]) : sin(th[k]);
        const double den = sj + sk;
        const double mjk = Kb[j + (long long)k * n], mkj = Kb[k + (long long)j * n];
        v = (den > 0.0) ? (mjk - mkj) / den : 0.0;
      }
      Kb[j + (long long)k * n] = v;
      Kb[k + (long long)j * n] = -v;
    }
  }
}

// The backward of `batch` problems with the two intermediates T and K (batch
// n x n blocks each, stride n*n) supplied by the caller.  Every element of T
// and K is written before it is read, so their previous contents do not matter.
static void csd_backward_ws(int batch, int n, const double* U1, const double* U2,
                            const double* V1, const double* theta, const double* g,
                            const double* G1, const double* G2, double* gA1, double* gA2,
                            double* T, double* K, hipStream_t s) {
  const long long nn = (long long)n * n;
  const double* U[2] = {U1, U2};
  const double* G[2] = {G1, G2};
  double* out[2] = {gA1, gA2};
  for (int blk = 0; blk < 2; ++blk) {
    GemmBatch base;
    base.batch = batch;
    base.m = n; base.n = n; base.k = n;
    if (G[blk]) {
      GemmBatch g1 = base;  // T = G V1
      g1.A = G[blk]; g1.lda = n; g1.sA = nn;
      g1.B = V1; g1.ldb = n; g1.sB = nn;
      g1.C = T; g1.ldc = n; g1.sC = nn;
      dgemm(g1, s);
      GemmBatch g2 = base;  // M = U^T T
      g2.transA = 1;
      g2.A = U[blk]; g2.lda = n; g2.sA = nn;
      g2.B = T; g2.ldb = n; g2.sB = nn;
      g2.C = K; g2.ldc = n; g2.sC = nn;
      dgemm(g2, s);
    }
    const long long npairs = (long long)n * (n + 1) / 2;
    const unsigned gx = (unsigned)std::max<long long>(1, std::min<long long>((npairs + 255) / 256, 4096));
    hipLaunchKernelGGL(csd_bwd_core_kernel, dim3(gx, batch), dim3(256), 0, s, n, K, nn, theta,
                       (long long)n, g, G[blk] ? 1 : 0, blk);
    ZCSD_CHECK_LAUNCH();
    GemmBatch g3 = base;  // T = U K
    g3.A = U[blk]; g3.lda = n; g3.sA = nn;
    g3.B = K; g3.ldb = n; g3.sB = nn;
    g3.C = T; g3.ldc = n; g3.sC = nn;
    dgemm(g3, s);
    GemmBatch g4 = base;  // gA = T V1^T
    g4.transB = 1;
    g4.A = T; g4.lda = n; g4.sA = nn;
    g4.B = V1; g4.ldb = n; g4.sB = nn;
    g4.C = out[blk]; g4.ldc = n; g4.sC = nn;
    dgemm(g4, s);
  }
}

void csd_backward(int batch, int n, const double* U1, const double* U2, const double* V1,
                  const double* theta, const double* g, const double* G1, const double* G2,
                  double* gA1, double* gA2, Arena& ar, hipStream_t s) {
  const long long nn = (long long)n * n;
  ArenaScope scope(ar);
  double* T = ar.dalloc((size_t)batch * nn);
  double* K = ar.dalloc((size_t)batch * nn);
  csd_backward_ws(batch, n, U1, U2, V1, theta, g, G1, G2, gA1, gA2, T, K, s);
}

// ---------------------------------------------------------------------------
// Allocation-free variant: T and K live in a file-scope device array of fixed
// size instead of the handle's arena.  Each device holds its own copy of the
// array (for as long as the process runs); host code reaches it only through
// the device address that hipGetSymbolAddress returns for the current device,
// looked up once per device when a handle is created.
constexpr long long kScratchDoubles = 1LL << 23;  // 64 MiB: 2 n^2 <= 2^23 for n <= 2048
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on `device`, which must be the current device.
double* backward_scratch(int device) {
  ZCSD_REQUIRE(device >= 0 && device < kMaxDevices, "backward scratch: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    ZCSD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ZCSD_REQUIRE(p != nullptr, "backward scratch: no device address");
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  return g_scratch_ptr[device];
}

}  // namespace zcsd

using namespace zcsd;

extern "C" zcsd_status zcsd_dcsd_backward(zcsd_handle* handle, int batch, int n, const double* d_U1,
                                          const double* d_U2, const double* d_V1,
                                          const double* d_theta, const double* d_g_theta,
                                          const double* d_G_W1, const double* d_G_W2, double* d_gA1,
                                          double* d_gA2) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(batch >= 1 && n >= 1, "csd_backward: batch and n must be positive");
    ZCSD_REQUIRE(batch <= 65535, "csd_backward: batch <= 65535");
    ZCSD_REQUIRE(d_U1 && d_U2 && d_V1 && d_theta && d_gA1 && d_gA2, "csd_backward: NULL pointer");
    ZCSD_HIP(hipSetDevice(handle->device));
    handle->arena.reset();
    handle->arena.reserve((size_t)2 * batch * n * n * sizeof(double) + (16u << 20));
    csd_backward(batch, n, d_U1, d_U2, d_V1, d_theta, d_g_theta, d_G_W1, d_G_W2, d_gA1, d_gA2,
                 handle->arena, handle->stream);
    ZCSD_HIP(hipStreamSynchronize(handle->stream));
  });
}

extern "C" zcsd_status zcsd_dcsd_backward_noalloc(zcsd_handle* handle, int batch, int n,
                                                  const double* d_U1, const double* d_U2,
                                                  const double* d_V1, const double* d_theta,
                                                  const double* d_g_theta, const double* d_G_W1,
                                                  const double* d_G_W2, double* d_gA1,
                                                  double* d_gA2) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(batch >= 1 && n >= 1, "csd_backward_noalloc: batch and n must be positive");
    ZCSD_REQUIRE(2LL * n * n <= kScratchDoubles,
                 "csd_backward_noalloc: n exceeds the scratch limit (2 n^2 <= 2^23 doubles, n <= 2048)");
    ZCSD_REQUIRE(d_U1 && d_U2 && d_V1 && d_theta && d_gA1 && d_gA2,
                 "csd_backward_noalloc: NULL pointer");
    ZCSD_HIP(hipSetDevice(handle->device));
    double* ptr = backward_scratch(handle->device);
    const long long nn = (long long)n * n;
    // problems per pass: T and K of every problem of the pass fit the array
    const int per = (int)std::min<long long>(std::min<long long>(kScratchDoubles / (2 * nn), 65535),
                                             batch);
    for (int b0 = 0; b0 < batch; b0 += per) {
      const int nb = std::min(per, batch - b0);
      const long long o = (long long)b0 * nn, ot = (long long)b0 * n;
      csd_backward_ws(nb, n, d_U1 + o, d_U2 + o, d_V1 + o, d_theta + ot,
                      d_g_theta ? d_g_theta + ot : nullptr, d_G_W1 ? d_G_W1 + o : nullptr,
                      d_G_W2 ? d_G_W2 + o : nullptr, d_gA1 + o, d_gA2 + o, ptr,
                      ptr + (long long)nb * nn, handle->stream);
    }
  });
}
