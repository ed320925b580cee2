// Internal declarations of libzcsd (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/zcsd.h"

namespace zcsd {

// ---------------------------------------------------------------------------
// errors
struct HipError : std::runtime_error {
  explicit HipError(const std::string& s) : std::runtime_error(s) {}
};
struct ArgError : std::runtime_error {
  explicit ArgError(const std::string& s) : std::runtime_error(s) {}
};
struct NumError : std::runtime_error {
  zcsd_status code;
  NumError(zcsd_status c, const std::string& s) : std::runtime_error(s), code(c) {}
};

#define ZCSD_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      throw ::zcsd::HipError(std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define ZCSD_CHECK_LAUNCH() ZCSD_HIP(hipGetLastError())

#define ZCSD_REQUIRE(cond, msg)                                                     \
  do {                                                                              \
    if (!(cond)) throw ::zcsd::ArgError(msg);                                       \
  } while (0)

// ---------------------------------------------------------------------------
// device workspace: a bump allocator over one hipMalloc'd block that grows
// between calls; every allocation is 256-byte aligned.
class Arena {
 public:
  ~Arena();
  void reserve(size_t bytes);      // make capacity >= bytes (frees and reallocates if needed)
  void reset() { top_ = 0; }
  size_t mark() const { return top_; }
  void release(size_t m) { top_ = m; }
  double* dalloc(size_t count) { return static_cast<double*>(alloc(count * sizeof(double))); }
  int* ialloc(size_t count) { return static_cast<int*>(alloc(count * sizeof(int))); }
  void* alloc(size_t bytes);
  size_t capacity() const { return cap_; }
  size_t high_water() const { return high_; }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, top_ = 0, high_ = 0;
};

// Scoped release of arena allocations made inside a block.
struct ArenaScope {
  Arena& a;
  size_t m;
  explicit ArenaScope(Arena& ar) : a(ar), m(ar.mark()) {}
  ~ArenaScope() { a.release(m); }
};

}  // namespace zcsd

namespace zcsd {
// default of the GEMM tiling threshold (GemmTileScope): two 128 x 128 tiles
// per compute unit
constexpr int kGemmTile128MinDefault = 512;
// One worker of the batched path: its own stream (default priority), its own
// second stream for overlapped side work, and its own workspace arena.
struct BatchWorker {
  hipStream_t stream = nullptr;
  hipStream_t aux = nullptr;
  Arena arena;
  ~BatchWorker();
};
}  // namespace zcsd

struct zcsd_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  zcsd::Arena arena;
  // the batched path's workers: the default number made with the handle,
  // more on a batched call whose tuning asks for them
  std::vector<std::unique_ptr<zcsd::BatchWorker>> workers;
  // pinned host staging for small readbacks
  double* h_stage = nullptr;
  size_t h_stage_count = 0;
  // batched-path tuning (zcsd_set_tuning): concurrent worker streams, and the
  // size-class steps for n <= 64, 64 < n <= 256 and n > 256
  int tune_workers = 4;
  int tune_step[3] = {8, 16, 64};
  // full-rank problems with n up to this run as whole CSDs of one workgroup
  // each, in persistent launches (0: none)
  int tune_small_max = 56;
  // products with at least this many 128 x 128 output tiles use that tiling
  int tune_tile128_min = zcsd::kGemmTile128MinDefault;
};

namespace zcsd {

// ---------------------------------------------------------------------------
// GEMM (gemm.hip).  Column-major, C_b = alpha_b op(A_b) op(B_b) + beta_b C_b.
struct GemmBatch {
  int transA = 0, transB = 0;
  int m = 0, n = 0, k = 0;
  const double* A = nullptr; long long lda = 0, sA = 0;
  const double* B = nullptr; long long ldb = 0, sB = 0;
  double* C = nullptr; long long ldc = 0, sC = 0;
  double alpha = 1.0, beta = 0.0;
  int batch = 1;
  // optional second batch dimension: problem (b1, b2) uses offsets b1*s? + b2*s?2
  int batch2 = 1;
  long long sA2 = 0, sB2 = 0, sC2 = 0;
  // optional workspace for split-K (deterministic: partial products, then a reduction)
  double* ws = nullptr;
  size_t ws_elems = 0;
  // symmetric product (m == n, beta == 0): only the tiles on or above the
  // diagonal are computed; the caller mirrors the upper triangle (mirror_upper)
  bool sym_upper = false;
  // only the upper triangle of C is wanted (m == n, any beta): the tiles below
  // the diagonal are skipped and keep their contents (no split-K)
  bool upper_only = false;
  // triangular operands (products known to be zero are skipped): K is made of
  // k / kseg segments, and within each segment op(A) is upper (tri & 1: zero
  // for k < i) or lower (tri & 2: zero for k > i), op(B) upper (tri & 4: zero
  // for k > j) or lower (tri & 8: zero for k < j), with k counted from the
  // segment start; the zeros must be present in memory
  int tri = 0, kseg = 0;
};
void dgemm(const GemmBatch& g, hipStream_t s);

// While a GemmLowpScope(true) is alive on this host thread, dgemm runs
// products on the FP32 matrix cores (FP64 operands rounded to FP32, FP32
// accumulation, FP64 result): every product when `always`, otherwise those
// where the FP32 instructions measured faster than FP64 (the demoted steps of
// the mixed-precision mode; gemm.hip).
class GemmLowpScope {
 public:
  explicit GemmLowpScope(bool on, bool always = false);
  ~GemmLowpScope();
  GemmLowpScope(const GemmLowpScope&) = delete;
  GemmLowpScope& operator=(const GemmLowpScope&) = delete;

 private:
  bool on_;
  int saved_;
};
// Inside a GemmLowpScope: products that must stay FP64 (the compact-WY factor of
// a blocked QR, whose orthogonality would otherwise degrade to the FP32 level)
class GemmFp64Scope {
 public:
  explicit GemmFp64Scope(bool on = true);
  ~GemmFp64Scope();
  GemmFp64Scope(const GemmFp64Scope&) = delete;
  GemmFp64Scope& operator=(const GemmFp64Scope&) = delete;

 private:
  bool on_;
  int saved_;
};
bool gemm_lowp_active();
// While a GemmTileScope(t) is alive on this host thread, products with at
// least t output tiles of 128 x 128 (over the batch) use that tiling and the
// others 64 x 64 tiles (default kGemmTile128MinDefault; a handle's
// ZCSD_TUNE_GEMM_TILE128_MIN, set for each call of the library)
class GemmTileScope {
 public:
  explicit GemmTileScope(int min_tiles);
  ~GemmTileScope();
  GemmTileScope(const GemmTileScope&) = delete;
  GemmTileScope& operator=(const GemmTileScope&) = delete;

 private:
  int saved_;
};
// products launched on the FP32 matrix cores by this host thread so far
long long gemm_lowp_launches();

// ---------------------------------------------------------------------------
// element-wise and reduction kernels (elem.hip)
// Y_b = alpha X_b (+ diag_add on the diagonal), m x n, per-batch strides.
void copy_scale(int batch, int m, int n, double alpha, const double* X, long long ldx, long long sx,
                double* Y, long long ldy, long long sy, hipStream_t s);
void add_diag(int batch, int n, double v, double* X, long long ldx, long long sx, hipStream_t s);
// Y = a X + b Y over `total` contiguous elements
void axpby(long long total, double a, const double* X, double b, double* Y, hipStream_t s);
void set_identity(int batch, int m, int n, double v, double* X, long long ldx, long long sx,
                  hipStream_t s);
// X_b = (X_b + X_b^T) / 2 in place (n x n)
void symmetrize(int batch, int n, double* X, long long ldx, long long sx, hipStream_t s);
// X_b(i, j) = X_b(j, i) for i > j (n x n): completes a sym_upper product
void mirror_upper(int batch, int n, double* X, long long ldx, long long sx, hipStream_t s);
// Sums of squares over a region of each X_b, reduced by many workgroups into
// per-problem partials and then in a fixed order (deterministic).
struct SumsqRegion {
  int m = 0, n = 0;               // rows x cols of every problem when nb is null
  const int* nb = nullptr;        // device: per-problem square extent n_b x n_b
  const int* np = nullptr;        // device, with nb: rows [np_b, n_b) x cols [0, np_b)
  const double* shift = nullptr;  // device, with nb: shift_b subtracted on the diagonal
  int max_cols = 0;               // with nb: an upper bound of the column extent
};
void sumsq_region(int batch, const double* X, long long ldx, long long sx, const SumsqRegion& r,
                  double* out, Arena& ar, hipStream_t s);
// out[b] = sum of squares of X_b (m x n) -> device array (length batch)
void sumsq(int batch, int m, int n, const double* X, long long ldx, long long sx, double* out,
           Arena& ar, hipStream_t s);

// ---------------------------------------------------------------------------
// host helpers
struct HostSync {
  static void sync(hipStream_t s) { ZCSD_HIP(hipStreamSynchronize(s)); }
};
void d2h(void* h, const void* d, size_t bytes, hipStream_t s);  // async + sync

// A second stream for work that can overlap the launches queued on s: the
// constructor makes it wait for everything queued on s so far; join() makes s
// wait for everything queued on it since.  One such stream per device, created
// on first use with the default priority.  The destructor joins when join()
// was not called (error paths), so later work on s stays ordered after it;
// memory that the side work uses must stay allocated until the join.
// The second stream that AuxStream uses on this host thread: `aux` from now on
// (nullptr: back to the device's shared one).  The batched path's workers
// each bring their own, so that their side work does not queue behind
// another worker's.
void set_thread_aux_stream(hipStream_t aux);
class AuxStream {
 public:
  explicit AuxStream(hipStream_t s);
  ~AuxStream();
  AuxStream(const AuxStream&) = delete;
  AuxStream& operator=(const AuxStream&) = delete;
  hipStream_t get() const { return aux_; }
  void join();

 private:
  hipStream_t s_ = nullptr, aux_ = nullptr;
  hipEvent_t fork_ = nullptr, done_ = nullptr;
  bool joined_ = false;
};
void h2d(void* d, const void* h, size_t bytes, hipStream_t s);  // queued on s (small: pinned staging, no wait)

// One problem of a batch through the single-problem CSD (csd.hip), with
// Algorithm 2: square blocks with ld n, outputs U1, U2, V1 (n x n, ld n) and
// theta (n) on the device; returns the rank and whether Algorithm 2 replaced
// a polar factor.  Needs csd_workspace_bytes(n) free in the arena.
int csd_single_member(int n, const double* A1, const double* A2, double* U1, double* U2,
                      double* V1, double* theta, const zcsd_opts& o, Arena& ar, hipStream_t s,
                      bool* repaired);
size_t csd_workspace_bytes(int n);
// the batched path's first W worker streams of a handle (csd_batched.hip)
void ensure_batch_workers(zcsd_handle_s* h, int W);
// whole CSDs of small full-rank problems, one workgroup each, in persistent
// launches (csd_small.hip), one per tier of sizes: small_csd_tiers gives the
// tiers' largest sizes (descending, the first is the largest size taken) and
// workgroups per compute unit, and returns their number (4);
// small_csd_scratch_bytes the global scratch for grids of grid[t] workgroups;
// small_csd_launch runs a list sorted by descending size whose first
// tier_count[0] entries belong to tier 0, the next tier_count[1] to tier 1 and
// so on.  status[t] of list entry t: low byte 0 = written, 1 = the l estimate
// reached eps, 2 = a Cholesky factorization broke down (1 and 2: nothing
// written); bits 8.. the Zolotarev degree used
int small_csd_tiers(int* max_n, int* per_cu);
size_t small_csd_scratch_bytes(const int* grid);
void small_csd_launch(const int* tier_count, const int* d_list, const int* d_n, const long long* d_off,
                      const long long* d_toff, const double* A1, const double* A2, double* U1,
                      double* U2, double* V1, double* theta, double eps, double tol,
                      bool theta_from_lambda, const int* grid, double* scratch, int* d_status, Arena& ar,
                      hipStream_t s);
// the same CSDs routed on the device (zcsd_dcsd_batched_small):
// small_table_device_make uploads the coefficient table of (eps, tol) for
// `device` once (synchronous; false if it was there);
// small_device_ws_bytes is the workspace of a batch of `batch` on n_cu compute
// units; small_device_launch enqueues the sort by size and the four
// persistent launches on s, with no host transfer, synchronisation or
// allocation.  status[k] of problem k as above, or 3 for a size outside 1..64.
bool small_table_device_make(int device, double eps, double tol);
size_t small_device_ws_bytes(int batch, int n_cu);
void small_device_launch(int device, int batch, const int* d_n, const long long* d_off,
                         const long long* d_toff, const double* A1, const double* A2, double* U1,
                         double* U2, double* V1, double* theta, double eps, double tol,
                         bool theta_from_lambda, int n_cu, void* ws, int* d_status, hipStream_t s);
// Householder QR of the m x n block A (m >= n, ld lda): Q (m x n, ld m) and
// the triangular R (n x n, ld n, zeros below the diagonal) (csd.hip)
void tall_qr(int m, int n, const double* A, long long lda, double* Q, double* R, Arena& ar,
             hipStream_t s);

// Device address of the fixed scratch array of the allocation-free backward
// (backward.hip) on `device`, which must be current; looked up once per device.
double* backward_scratch(int device);

}  // namespace zcsd
