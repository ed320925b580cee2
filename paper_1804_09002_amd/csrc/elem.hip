// Element-wise and reduction kernels (HBM-bound helpers around the MFMA path)
// and the device workspace arena.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>

#include "zcsd_internal.h"
#include "zcsd_la.h"

namespace zcsd {

// ---------------------------------------------------------------------------
// Arena
Arena::~Arena() {
  if (base_) (void)hipFree(base_);
}

void Arena::reserve(size_t bytes) {
  if (bytes <= cap_) return;
  if (top_ != 0) throw HipError("arena: reserve while allocations are live");
  if (base_) {
    ZCSD_HIP(hipDeviceSynchronize());
    ZCSD_HIP(hipFree(base_));
    base_ = nullptr;
    cap_ = 0;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw NumError(ZCSD_ENOMEM, "arena: hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  base_ = static_cast<char*>(p);
  cap_ = bytes;
}

void* Arena::alloc(size_t bytes) {
  size_t off = (top_ + 255) & ~size_t(255);
  if (off + bytes > cap_)
    throw NumError(ZCSD_ENOMEM, "arena: out of workspace (need " + std::to_string(off + bytes) +
                                    ", have " + std::to_string(cap_) + ")");
  top_ = off + bytes;
  high_ = std::max(high_, top_);
  return base_ + off;
}

// Small transfers from or to pageable host memory.  A copy from pageable
// memory is not guaranteed to wait for kernels already queued on the stream,
// and the destination of an upload is often arena memory that a queued kernel
// still reads (arena blocks are reused as soon as a scope ends), so the stream
// is drained before and after such a copy.  Transfers of at most kSlotBytes
// go instead through a ring of pinned staging slots per stream: an upload is
// copied into a slot on the host and the slot's copy to the device is queued
// on the stream (ordered after the kernels before it, so the arena hazard is
// covered by the stream order), with no host wait, and an event recorded
// after the copy guards the slot's reuse; a download is queued into a slot,
// waited for once, and copied out on the host.
namespace {
constexpr int kSlots = 64;
constexpr size_t kSlotBytes = (size_t)64 << 10;
struct UploadRing {
  std::mutex mu;
  char* host = nullptr;  // kSlots x kSlotBytes, pinned
  hipEvent_t ev[kSlots] = {};
  bool pending[kSlots] = {};
  int next = 0;
};
// one ring per stream, kept to the end of the process (a stream value reused
// by a later stream reuses the ring, whose slots are guarded by their events)
UploadRing* ring_for(hipStream_t s) {
  static std::mutex mu;
  static std::map<hipStream_t, UploadRing*> rings;
  std::lock_guard<std::mutex> g(mu);
  auto it = rings.find(s);
  if (it != rings.end()) return it->second;
  auto* r = new UploadRing();
  void* p = nullptr;
  if (hipHostMalloc(&p, kSlots * kSlotBytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    delete r;
    return nullptr;
  }
  r->host = static_cast<char*>(p);
  for (int k = 0; k < kSlots; ++k) ZCSD_HIP(hipEventCreateWithFlags(&r->ev[k], hipEventDisableTiming));
  rings[s] = r;
  return r;
}
}  // namespace

void d2h(void* h, const void* d, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  if (bytes <= kSlotBytes) {
    if (UploadRing* r = ring_for(s)) {
      // into a pinned slot: the copy is ordered after the kernels before it,
      // and one wait for it replaces the drain before and the wait after
      std::lock_guard<std::mutex> g(r->mu);
      const int k = r->next;
      r->next = (k + 1) % kSlots;
      if (r->pending[k]) ZCSD_HIP(hipEventSynchronize(r->ev[k]));
      char* slot = r->host + (size_t)k * kSlotBytes;
      ZCSD_HIP(hipMemcpyAsync(slot, d, bytes, hipMemcpyDeviceToHost, s));
      ZCSD_HIP(hipEventRecord(r->ev[k], s));
      ZCSD_HIP(hipEventSynchronize(r->ev[k]));
      r->pending[k] = false;
      std::memcpy(h, slot, bytes);
      return;
    }
  }
  ZCSD_HIP(hipStreamSynchronize(s));
  ZCSD_HIP(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s));
  ZCSD_HIP(hipStreamSynchronize(s));
}

void h2d(void* d, const void* h, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  if (bytes <= kSlotBytes) {
    if (UploadRing* r = ring_for(s)) {
      std::lock_guard<std::mutex> g(r->mu);
      const int k = r->next;
      r->next = (k + 1) % kSlots;
      if (r->pending[k]) ZCSD_HIP(hipEventSynchronize(r->ev[k]));
      char* slot = r->host + (size_t)k * kSlotBytes;
      std::memcpy(slot, h, bytes);
      ZCSD_HIP(hipMemcpyAsync(d, slot, bytes, hipMemcpyHostToDevice, s));
      ZCSD_HIP(hipEventRecord(r->ev[k], s));
      r->pending[k] = true;
      return;
    }
  }
  ZCSD_HIP(hipStreamSynchronize(s));
  ZCSD_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
  ZCSD_HIP(hipStreamSynchronize(s));
}

namespace {
thread_local hipStream_t g_aux_override = nullptr;
}
void set_thread_aux_stream(hipStream_t aux) { g_aux_override = aux; }

BatchWorker::~BatchWorker() {
  if (stream) (void)hipStreamDestroy(stream);
  if (aux) (void)hipStreamDestroy(aux);
}

static hipStream_t aux_stream_for_current_device() {
  if (g_aux_override) return g_aux_override;
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  ZCSD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t st = nullptr;
  ZCSD_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  streams[dev] = st;
  return st;
}

AuxStream::AuxStream(hipStream_t s) : s_(s) {
  aux_ = aux_stream_for_current_device();
  ZCSD_HIP(hipEventCreateWithFlags(&fork_, hipEventDisableTiming));
  ZCSD_HIP(hipEventCreateWithFlags(&done_, hipEventDisableTiming));
  ZCSD_HIP(hipEventRecord(fork_, s_));
  ZCSD_HIP(hipStreamWaitEvent(aux_, fork_, 0));
}

void AuxStream::join() {
  if (joined_) return;
  joined_ = true;
  ZCSD_HIP(hipEventRecord(done_, aux_));
  ZCSD_HIP(hipStreamWaitEvent(s_, done_, 0));
}

AuxStream::~AuxStream() {
  if (!joined_) {
    joined_ = true;
    if (hipEventRecord(done_, aux_) != hipSuccess || hipStreamWaitEvent(s_, done_, 0) != hipSuccess)
      (void)hipStreamSynchronize(aux_);
  }
  (void)hipEventDestroy(fork_);
  (void)hipEventDestroy(done_);
}

// ---------------------------------------------------------------------------
// kernels: grid = (ceil(m*n / 256) capped, batch); element e -> (i, j) with i fastest

__global__ void copy_scale_kernel(int m, int n, double alpha, const double* __restrict__ X,
                                  long long ldx, long long sx, double* Y, long long ldy,
                                  long long sy) {
  const long long b = blockIdx.y;
  const long long total = (long long)m * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    Y[b * sy + i + j * ldy] = alpha * X[b * sx + i + j * ldx];
  }
}

__global__ void add_diag_kernel(int n, double v, double* X, long long ldx, long long sx) {
  const long long b = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    X[b * sx + i + (long long)i * ldx] += v;
}

__global__ void set_identity_kernel(int m, int n, double v, double* X, long long ldx,
                                    long long sx) {
  const long long b = blockIdx.y;
  const long long total = (long long)m * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    X[b * sx + i + j * ldx] = (i == j) ? v : 0.0;
  }
}

__global__ void set_identity_scaled_kernel(int m, int n, const double* vals, double v, double* X,
                                           long long ldx, long long sx) {
  const long long b = blockIdx.y;
  const double d = vals ? vals[b] : v;
  const long long total = (long long)m * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    X[b * sx + i + j * ldx] = (i == j) ? d : 0.0;
  }
}

// (X + X^T)/2 in place: thread handles (i, j) with i > j and writes both
__global__ void symmetrize_kernel(int n, double* X, long long ldx, long long sx) {
  const long long b = blockIdx.y;
  const long long total = (long long)n * n;
  double* Xb = X + b * sx;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    if (i > j) {
      const double v = 0.5 * (Xb[i + (long long)j * ldx] + Xb[j + (long long)i * ldx]);
      Xb[i + (long long)j * ldx] = v;
      Xb[j + (long long)i * ldx] = v;
    }
  }
}

// per-batch sum of squares; grid (1, batch), block 256, two-level reduction
// partial[b * G + g] = sum over the columns j = c0 + g, c0 + g + G, ... of the
// region of X_b; every workgroup walks whole columns (coalesced rows).
__global__ void sumsq_partial_kernel(const double* __restrict__ X, long long ldx, long long sx,
                                     SumsqRegion R, int G, double* part) {
  const int b = blockIdx.y, g = blockIdx.x;
  int r0 = 0, r1 = R.m, c0 = 0, c1 = R.n;
  double sh = 0.0;
  if (R.nb) {
    const int m = R.nb[b];
    r1 = m;
    c1 = m;
    if (R.np) {
      r0 = R.np[b];
      c1 = r0;
    }
    if (R.shift) sh = R.shift[b];
  }
  const double* Xb = X + (long long)b * sx;
  double acc = 0.0;
  for (int j = c0 + g; j < c1; j += G)
    for (int i = r0 + (int)threadIdx.x; i < r1; i += blockDim.x) {
      const double v = Xb[i + (long long)j * ldx] - (i == j ? sh : 0.0);
      acc += v * v;
    }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)b * G + g] = red[0];
}

// out[b] = sum of the G partials of problem b, in a fixed order
__global__ void sumsq_final_kernel(int G, const double* __restrict__ part, double* out) {
  const int b = blockIdx.x;
  double acc = 0.0;
  for (int g = threadIdx.x; g < G; g += blockDim.x) acc += part[(long long)b * G + g];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = red[0];
}

static dim3 egrid(long long total, int batch) {
  long long g = (total + 255) / 256;
  g = std::max<long long>(1, std::min<long long>(g, 4096));
  return dim3((unsigned)g, (unsigned)batch);
}

void copy_scale(int batch, int m, int n, double alpha, const double* X, long long ldx,
                long long sx, double* Y, long long ldy, long long sy, hipStream_t s) {
  if (batch <= 0 || m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(copy_scale_kernel, egrid((long long)m * n, batch), dim3(256), 0, s, m, n,
                     alpha, X, ldx, sx, Y, ldy, sy);
  ZCSD_CHECK_LAUNCH();
}

// Y = a X + b Y over contiguous elements
__global__ void axpby_kernel(long long total, double a, const double* __restrict__ X, double b,
                             double* Y) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x)
    Y[e] = a * X[e] + b * Y[e];
}

void axpby(long long total, double a, const double* X, double b, double* Y, hipStream_t s) {
  if (total <= 0) return;
  const long long g = std::max<long long>(1, std::min<long long>((total + 255) / 256, 4096));
  hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)g), dim3(256), 0, s, total, a, X, b, Y);
  ZCSD_CHECK_LAUNCH();
}

void add_diag(int batch, int n, double v, double* X, long long ldx, long long sx, hipStream_t s) {
  if (batch <= 0 || n <= 0) return;
  hipLaunchKernelGGL(add_diag_kernel, egrid(n, batch), dim3(256), 0, s, n, v, X, ldx, sx);
  ZCSD_CHECK_LAUNCH();
}

void set_identity(int batch, int m, int n, double v, double* X, long long ldx, long long sx,
                  hipStream_t s) {
  if (batch <= 0 || m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(set_identity_kernel, egrid((long long)m * n, batch), dim3(256), 0, s, m, n,
                     v, X, ldx, sx);
  ZCSD_CHECK_LAUNCH();
}

void set_identity_scaled(int batch, int m, int n, const double* d_vals, double v, double* X,
                         long long ldx, long long sx, hipStream_t s) {
  if (batch <= 0 || m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(set_identity_scaled_kernel, egrid((long long)m * n, batch), dim3(256), 0, s,
                     m, n, d_vals, v, X, ldx, sx);
  ZCSD_CHECK_LAUNCH();
}

void symmetrize(int batch, int n, double* X, long long ldx, long long sx, hipStream_t s) {
  if (batch <= 0 || n <= 0) return;
  hipLaunchKernelGGL(symmetrize_kernel, egrid((long long)n * n, batch), dim3(256), 0, s, n, X,
                     ldx, sx);
  ZCSD_CHECK_LAUNCH();
}

__global__ void mirror_upper_kernel(int n, double* X, long long ldx, long long sx) {
  const long long b = blockIdx.y;
  const long long total = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    if (i > j) X[b * sx + i + (long long)j * ldx] = X[b * sx + j + (long long)i * ldx];
  }
}

void mirror_upper(int batch, int n, double* X, long long ldx, long long sx, hipStream_t s) {
  if (batch <= 0 || n <= 0) return;
  hipLaunchKernelGGL(mirror_upper_kernel, egrid((long long)n * n, batch), dim3(256), 0, s, n, X,
                     ldx, sx);
  ZCSD_CHECK_LAUNCH();
}

void sumsq_region(int batch, const double* X, long long ldx, long long sx, const SumsqRegion& r,
                  double* out, Arena& ar, hipStream_t s) {
  if (batch <= 0) return;
  const int cols = r.nb ? r.max_cols : r.n;
  ZCSD_REQUIRE(batch <= 65535, "sumsq: batch <= 65535");
  const int G = std::max(1, std::min(cols, std::max(1, 2048 / batch)));
  ArenaScope sc(ar);
  double* part = ar.dalloc((size_t)batch * G);
  hipLaunchKernelGGL(sumsq_partial_kernel, dim3(G, batch), dim3(256), 0, s, X, ldx, sx, r, G, part);
  ZCSD_CHECK_LAUNCH();
  hipLaunchKernelGGL(sumsq_final_kernel, dim3(batch), dim3(256), 0, s, G, part, out);
  ZCSD_CHECK_LAUNCH();
}

void sumsq(int batch, int m, int n, const double* X, long long ldx, long long sx, double* out,
           Arena& ar, hipStream_t s) {
  SumsqRegion r;
  r.m = m;
  r.n = n;
  sumsq_region(batch, X, ldx, sx, r, out, ar, s);
}

}  // namespace zcsd
