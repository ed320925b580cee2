// Element-wise and reduction kernels (HBM-bound helpers around the MFMA path)
// and the device workspace arena.
#include <algorithm>

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

void d2h(void* h, const void* d, size_t bytes, hipStream_t s) {
  ZCSD_HIP(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s));
  ZCSD_HIP(hipStreamSynchronize(s));
}

void h2d(void* d, const void* h, size_t bytes, hipStream_t s) {
  ZCSD_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
  ZCSD_HIP(hipStreamSynchronize(s));
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
__global__ void sumsq_kernel(int m, int n, const double* __restrict__ X, long long ldx,
                             long long sx, double* out) {
  const long long b = blockIdx.y;
  const long long total = (long long)m * n;
  double acc = 0.0;
  for (long long e = threadIdx.x; e < total; e += blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    const double v = X[b * sx + i + j * ldx];
    acc += v * v;
  }
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

void sumsq(int batch, int m, int n, const double* X, long long ldx, long long sx, double* out,
           hipStream_t s) {
  if (batch <= 0) return;
  hipLaunchKernelGGL(sumsq_kernel, dim3(1, batch), dim3(256), 0, s, m, n, X, ldx, sx, out);
  ZCSD_CHECK_LAUNCH();
}

}  // namespace zcsd
