// C ABI entry points: handle management, option defaults, status strings and
// the exception-to-status boundary shared by every entry point.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "zcsd_api_guard.h"
#include "zcsd_internal.h"
#include "zcsd_la.h"

using namespace zcsd;

extern "C" {

zcsd_status zcsd_create(zcsd_handle** handle, int device) {
  if (!handle) return ZCSD_EINVAL;
  *handle = nullptr;
  return guarded([&] {
    int count = 0;
    ZCSD_HIP(hipGetDeviceCount(&count));
    ZCSD_REQUIRE(device >= 0 && device < count, "zcsd_create: no such device");
    ZCSD_HIP(hipSetDevice(device));
    // the allocation-free entry point's scratch array: its address on this
    // device, looked up here once so that the entry point itself makes no
    // runtime call beyond its kernel launches
    (void)backward_scratch(device);
    auto* h = new zcsd_handle_s();
    h->device = device;
    h->stream = nullptr;
    h->h_stage_count = 1 << 16;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h->h_stage),
                                 h->h_stage_count * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
      delete h;
      ZCSD_HIP(e);
    }
    // the batched path's worker streams, made here rather than on its first
    // call: the runtime spreads streams over its few hardware queues in
    // creation order, and created before any other stream of the library
    // they get the same queues in every process (made after the single
    // path's second stream, two workers shared a queue: 2048 ragged problems
    // took 0.142 instead of 0.112 s)
    try {
      ensure_batch_workers(h, h->tune_workers);
    } catch (...) {
      (void)hipHostFree(h->h_stage);
      delete h;
      throw;
    }
    *handle = h;
  });
}

zcsd_status zcsd_destroy(zcsd_handle* handle) {
  if (!handle) return ZCSD_OK;
  return guarded([&] {
    ZCSD_HIP(hipSetDevice(handle->device));
    ZCSD_HIP(hipDeviceSynchronize());
    if (handle->h_stage) (void)hipHostFree(handle->h_stage);
    delete handle;
  });
}

zcsd_status zcsd_set_stream(zcsd_handle* handle, void* stream) {
  if (!handle) return ZCSD_EINVAL;
  handle->stream = static_cast<hipStream_t>(stream);
  return ZCSD_OK;
}

zcsd_status zcsd_set_tuning(zcsd_handle* handle, int key, int value) {
  if (!handle) return ZCSD_EINVAL;
  switch (key) {
    case ZCSD_TUNE_BATCHED_WORKERS:
      if (value < 1 || value > 16) return ZCSD_EINVAL;
      handle->tune_workers = value;
      return ZCSD_OK;
    case ZCSD_TUNE_CLASS_STEP_SMALL:
    case ZCSD_TUNE_CLASS_STEP_MID:
    case ZCSD_TUNE_CLASS_STEP_LARGE:
      if (value < 1 || value > 256) return ZCSD_EINVAL;
      handle->tune_step[key - ZCSD_TUNE_CLASS_STEP_SMALL] = value;
      return ZCSD_OK;
    case ZCSD_TUNE_ONE_WORKGROUP_MAX_N:
      {
        int mx[8];
        zcsd::small_csd_tiers(mx, nullptr);
        if (value < 0 || value > mx[0]) return ZCSD_EINVAL;
      }
      handle->tune_small_max = value;
      return ZCSD_OK;
    case ZCSD_TUNE_GEMM_TILE128_MIN:
      if (value < 1 || value > (1 << 24)) return ZCSD_EINVAL;
      handle->tune_tile128_min = value;
      return ZCSD_OK;
    default:
      return ZCSD_EINVAL;
  }
}

zcsd_status zcsd_get_tuning(zcsd_handle* handle, int key, int* value) {
  if (!handle || !value) return ZCSD_EINVAL;
  switch (key) {
    case ZCSD_TUNE_BATCHED_WORKERS:
      *value = handle->tune_workers;
      return ZCSD_OK;
    case ZCSD_TUNE_CLASS_STEP_SMALL:
    case ZCSD_TUNE_CLASS_STEP_MID:
    case ZCSD_TUNE_CLASS_STEP_LARGE:
      *value = handle->tune_step[key - ZCSD_TUNE_CLASS_STEP_SMALL];
      return ZCSD_OK;
    case ZCSD_TUNE_ONE_WORKGROUP_MAX_N:
      *value = handle->tune_small_max;
      return ZCSD_OK;
    case ZCSD_TUNE_GEMM_TILE128_MIN:
      *value = handle->tune_tile128_min;
      return ZCSD_OK;
    default:
      return ZCSD_EINVAL;
  }
}

size_t zcsd_sizeof_opts(void) { return sizeof(zcsd_opts); }
size_t zcsd_sizeof_info(void) { return sizeof(zcsd_info); }

void zcsd_default_opts(zcsd_opts* o) {
  if (!o) return;
  o->prec = ZCSD_FP64;
  o->rank_mode = ZCSD_RANK_AUTO;
  o->eps = 1e-15;
  o->mu = 2.0;
  o->tol = std::ldexp(1.0, -53);
  o->r_override = 0;
  o->ell_override = 0.0;
  o->n_leaf = 64;
  o->postprocess = 1;
}

const char* zcsd_status_string(zcsd_status s) {
  switch (s) {
    case ZCSD_OK: return "ZCSD_OK";
    case ZCSD_EINVAL: return "ZCSD_EINVAL: invalid argument";
    case ZCSD_ENOTISO: return "ZCSD_ENOTISO: input is not close to a partial isometry";
    case ZCSD_ENOCONV: return "ZCSD_ENOCONV: Zolotarev iteration or divide-and-conquer split did not converge";
    case ZCSD_EREPAIR: return "ZCSD_EREPAIR: ill-conditioned repair rejected";
    case ZCSD_EHIP: return "ZCSD_EHIP: HIP runtime error";
    case ZCSD_ENOMEM: return "ZCSD_ENOMEM: device allocation failed";
  }
  return "unknown zcsd_status";
}

zcsd_status zcsd_dgemm(zcsd_handle* handle, int transA, int transB, int m, int n, int k,
                       double alpha, const double* A, int lda, long long strideA, const double* B,
                       int ldb, long long strideB, double beta, double* C, int ldc,
                       long long strideC, int batch) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(m >= 0 && n >= 0 && k >= 0 && batch >= 0, "dgemm: negative size");
    if (m == 0 || n == 0 || batch == 0) return;
    ZCSD_REQUIRE(C && (k == 0 || (A && B)), "dgemm: NULL pointer");
    ZCSD_REQUIRE(ldc >= std::max(1, m), "dgemm: ldc too small");
    ZCSD_REQUIRE(k == 0 || (lda >= std::max(1, transA ? k : m) && ldb >= std::max(1, transB ? n : k)),
                 "dgemm: leading dimension too small");
    ZCSD_HIP(hipSetDevice(handle->device));
    GemmBatch g;
    g.transA = transA != 0;
    g.transB = transB != 0;
    g.m = m; g.n = n; g.k = k;
    g.A = A; g.lda = lda; g.sA = strideA;
    g.B = B; g.ldb = ldb; g.sB = strideB;
    g.C = C; g.ldc = ldc; g.sC = strideC;
    g.alpha = alpha; g.beta = beta; g.batch = batch;
    dgemm(g, handle->stream);
  });
}
zcsd_status zcsd_dgemm_f32acc(zcsd_handle* handle, int transA, int transB, int m, int n, int k,
                       double alpha, const double* A, int lda, long long strideA, const double* B,
                       int ldb, long long strideB, double beta, double* C, int ldc,
                       long long strideC, int batch) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(m >= 0 && n >= 0 && k >= 0 && batch >= 0, "dgemm_f32acc: negative size");
    if (m == 0 || n == 0 || batch == 0) return;
    ZCSD_REQUIRE(C && (k == 0 || (A && B)), "dgemm_f32acc: NULL pointer");
    ZCSD_REQUIRE(ldc >= std::max(1, m), "dgemm_f32acc: ldc too small");
    ZCSD_REQUIRE(k == 0 || (lda >= std::max(1, transA ? k : m) && ldb >= std::max(1, transB ? n : k)),
                 "dgemm_f32acc: leading dimension too small");
    ZCSD_HIP(hipSetDevice(handle->device));
    GemmBatch g;
    g.transA = transA != 0;
    g.transB = transB != 0;
    g.m = m; g.n = n; g.k = k;
    g.A = A; g.lda = lda; g.sA = strideA;
    g.B = B; g.ldb = ldb; g.sB = strideB;
    g.C = C; g.ldc = ldc; g.sC = strideC;
    g.alpha = alpha; g.beta = beta; g.batch = batch;
    GemmLowpScope lowp(true, /*always=*/true);
    dgemm(g, handle->stream);
  });
}

zcsd_status zcsd_dgemm_ex(zcsd_handle* handle, int transA, int transB, int m, int n, int k,
                          double alpha, const double* A, int lda, long long strideA,
                          const double* B, int ldb, long long strideB, double beta, double* C,
                          int ldc, long long strideC, int batch, int flags, int tri, int kseg,
                          double* d_ws, size_t ws_elems) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(m >= 0 && n >= 0 && k >= 0 && batch >= 0, "dgemm_ex: negative size");
    ZCSD_REQUIRE((flags & ~(ZCSD_GEMM_SYM_UPPER | ZCSD_GEMM_UPPER_ONLY | ZCSD_GEMM_F32ACC)) == 0,
                 "dgemm_ex: unknown flag");
    ZCSD_REQUIRE(tri >= 0 && tri <= 15 && kseg >= 0, "dgemm_ex: tri must be in 0..15");
    ZCSD_REQUIRE(!(d_ws == nullptr && ws_elems > 0), "dgemm_ex: ws_elems without a workspace");
    if (m == 0 || n == 0 || batch == 0) return;
    ZCSD_REQUIRE(C && (k == 0 || (A && B)), "dgemm_ex: NULL pointer");
    ZCSD_REQUIRE(ldc >= std::max(1, m), "dgemm_ex: ldc too small");
    ZCSD_REQUIRE(k == 0 || (lda >= std::max(1, transA ? k : m) && ldb >= std::max(1, transB ? n : k)),
                 "dgemm_ex: leading dimension too small");
    ZCSD_HIP(hipSetDevice(handle->device));
    GemmBatch g;
    g.transA = transA != 0;
    g.transB = transB != 0;
    g.m = m; g.n = n; g.k = k;
    g.A = A; g.lda = lda; g.sA = strideA;
    g.B = B; g.ldb = ldb; g.sB = strideB;
    g.C = C; g.ldc = ldc; g.sC = strideC;
    g.alpha = alpha; g.beta = beta; g.batch = batch;
    g.sym_upper = (flags & ZCSD_GEMM_SYM_UPPER) != 0;
    g.upper_only = (flags & ZCSD_GEMM_UPPER_ONLY) != 0;
    g.tri = tri;
    g.kseg = kseg;
    g.ws = d_ws;
    g.ws_elems = ws_elems;
    GemmLowpScope lowp((flags & ZCSD_GEMM_F32ACC) != 0, /*always=*/true);
    dgemm(g, handle->stream);
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
#include "zcsd_zolo.h"

namespace {
size_t zolo_pd_ws_bytes(int batch, int n) {
  const size_t nn = (size_t)n * n;
  // iterates and products, plus the two QR workspaces (at most 8 terms)
  return (size_t)batch * (64 * nn + 64 * (size_t)n) * sizeof(double) +
         qr_work_bytes(QRShape::General, batch, n, n, 32) +
         qr_work_bytes(QRShape::Stacked, 8 * batch, 2 * n, n, 32) + (64u << 20);
}
}  // namespace

extern "C" zcsd_status zcsd_dzolo_pd(zcsd_handle* handle, int batch, int n, double alpha,
                                     const double* d_X, int ldx, long long strideX, double* d_W,
                                     double* d_H, double* d_X1, const zcsd_opts* opts,
                                     zcsd_info* info) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(batch >= 1 && n >= 1, "zolo_pd: batch and n must be positive");
    ZCSD_REQUIRE(d_X && d_W, "zolo_pd: NULL pointer");
    ZCSD_REQUIRE(ldx >= n, "zolo_pd: ldx < n");
    ZCSD_REQUIRE(alpha > 0.0 && std::isfinite(alpha), "zolo_pd: alpha must be positive");
    zcsd_opts o;
    zcsd_default_opts(&o);
    if (opts) o = *opts;
    ZCSD_REQUIRE(o.r_override >= 0 && o.r_override <= ZOLO_RMAX, "zolo_pd: r_override out of range");
    ZCSD_HIP(hipSetDevice(handle->device));
    handle->arena.reset();
    handle->arena.reserve(zolo_pd_ws_bytes(batch, n));
    ZoloPdArgs a;
    a.batch = batch;
    a.n = n;
    a.alpha = alpha;
    a.X = d_X; a.ldx = ldx; a.sx = strideX;
    a.W = d_W; a.H = d_H; a.X1 = d_X1;
    a.eps = o.eps; a.tol = o.tol;
    a.r_override = o.r_override;
    a.ell_override = o.ell_override;
    ZoloPdResult r = zolo_pd_batched(a, handle->arena, handle->stream);
    ZCSD_HIP(hipStreamSynchronize(handle->stream));
    if (info) {
      *info = zcsd_info{};
      info->rank = n;
      info->r_used[0] = info->r_used[1] = r.r;
      info->ell[0] = info->ell[1] = r.ell;
      info->zolo_resid = r.resid;
    }
  });
}

extern "C" zcsd_status zcsd_dqr(zcsd_handle* handle, int batch, int stacked, int m, int n,
                                double* d_M, int ldm, long long strideM, double* d_Q, int ldq,
                                long long strideQ) {
  if (!handle) return ZCSD_EINVAL;
  return guarded([&] {
    GemmTileScope tile_scope(handle->tune_tile128_min);
    ZCSD_REQUIRE(batch >= 1 && n >= 1 && m >= n, "qr: need batch >= 1, m >= n >= 1");
    ZCSD_REQUIRE(!stacked || m == 2 * n, "qr: stacked shape needs m == 2n");
    ZCSD_REQUIRE(d_M && ldm >= m, "qr: bad M");
    ZCSD_REQUIRE(!d_Q || ldq >= m, "qr: bad Q");
    ZCSD_HIP(hipSetDevice(handle->device));
    const QRShape shape = stacked ? QRShape::Stacked : QRShape::General;
    const size_t need = qr_work_bytes(shape, batch, m, n, 32) + (16u << 20);
    handle->arena.reset();
    handle->arena.reserve(need);
    QRWork wk = qr_work_alloc(handle->arena, shape, batch, m, n, 32);
    geqrf_batched(batch, shape, m, n, d_M, ldm, strideM, wk, handle->stream);
    if (d_Q) orgqr_batched(batch, shape, m, n, d_Q, ldq, strideQ, nullptr, wk, handle->stream);
    ZCSD_HIP(hipStreamSynchronize(handle->stream));
  });
}
