// Blocked Householder QR on the gfx950 path (batched, FP64).
//
// Two shapes share one engine:
//  * General: an m x n matrix (m >= n).  Panel k (columns c0 = k*nb ..) acts on
//    rows [c0, m).
//  * Stacked: the 2n x n matrix [R; sqrt(c) I] of the QR form of a Zolotarev
//    term (Sec. 5), with R upper triangular.  Reflector j only touches top row
//    j and bottom rows 0..j (the bottom block fills in as an upper triangle),
//    so panel k acts on the two row segments top [c0, c0+w) and bottom
//    [n, n + c0 + w): the panels grow from 2w to n + w rows instead of a
//    constant 2n, and the factorisation costs ~2n^3/3 flops instead of 10n^3/3.
//
// Each panel is factored by one workgroup (qr_panel_kernel): the panel's rows
// are copied into a contiguous buffer V (logical rows: segment 1 then
// segment 2), Householder reflectors are computed column by column with
// workgroup reductions, and the compact-WY factor T (H_1...H_w = I - V T V^T)
// is built on the fly from the same reductions.  R goes back into the matrix,
// the annihilated entries become exact zeros.  Trailing updates and Q
// formation are MFMA GEMMs on the two segments.
#include <algorithm>
#include <cmath>

#include "zcsd_internal.h"
#include "zcsd_la.h"
#include "zcsd_prof.h"

namespace zcsd {

constexpr int QR_NT = 256;
// inner-panel update (two-level factorisation): panel width, most columns
// updated, rows per partial-product workgroup, rows staged per step, rows per
// apply workgroup
constexpr int PU_W = 32, PU_NC = 96, PU_CH = 256, PU_SUB = 64, PU_RT = 64;

template <int NW>
__device__ __forceinline__ void wave_sum_multi(double (&p)[NW]) {
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    double v = p[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    p[j] = v;
  }
}

// logical row -> physical row of the matrix
__device__ __forceinline__ int qr_phys(int i, int h1, int r1a, int r2a) {
  return i < h1 ? r1a + i : r2a + (i - h1);
}

template <int NB>
__global__ __launch_bounds__(QR_NT) void qr_panel_kernel(double* M, long long ldm, long long sM,
                                                         int c0, int w, int r1a, int r1b, int r2a,
                                                         int r2b, double* V, long long ldv,
                                                         long long sV, double* T, long long sT) {
  constexpr int NWV = QR_NT / 64;
  __shared__ double red[NWV][NB];
  __shared__ double sums[NB];
  __shared__ double Ts[NB][NB + 1];
  __shared__ double betas[NB];
  __shared__ double sig_sh;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long b = blockIdx.x;
  M += b * sM;
  V += b * sV;
  T += b * sT;
  const int h1 = r1b - r1a, h2 = r2b - r2a, h = h1 + h2;

  // copy the panel into V (logical rows)
  for (long long e = tid; e < (long long)h * w; e += QR_NT) {
    const int i = (int)(e % h), j = (int)(e / h);
    V[i + j * ldv] = M[qr_phys(i, h1, r1a, r2a) + (long long)(c0 + j) * ldm];
  }
  for (int e = tid; e < NB * (NB + 1); e += QR_NT) (&Ts[0][0])[e] = 0.0;
  __syncthreads();

  for (int t = 0; t < w; ++t) {
    double* vt = V + (long long)t * ldv;
    // ||x(t+1:h)||^2
    double p[1] = {0.0};
    for (int i = t + 1 + tid; i < h; i += QR_NT) {
      const double x = vt[i];
      p[0] += x * x;
    }
    wave_sum_multi<1>(p);
    if (lane == 0) red[wave][0] = p[0];
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int q = 0; q < NWV; ++q) s += red[q][0];
      sig_sh = s;
    }
    __syncthreads();
    const double sig2 = sig_sh;
    const double alpha = vt[t];
    double tau, beta, scal;
    if (sig2 == 0.0) {  // H = I (LAPACK convention: no reflection, R_tt = alpha)
      tau = 0.0;
      beta = alpha;
      scal = 1.0;
    } else {
      const double nrm = sqrt(alpha * alpha + sig2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    __syncthreads();  // every thread has read alpha
    if (tid == 0) {
      vt[t] = 1.0;
      betas[t] = beta;
    }
    for (int i = t + 1 + tid; i < h; i += QR_NT) vt[i] *= scal;
    __syncthreads();

    // d_j = V(t,j) + sum_{i>t} v_i V(i,j), j != t: the T column (j < t) and the update (j > t)
    double d[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) d[j] = 0.0;
    for (int i = t + 1 + tid; i < h; i += QR_NT) {
      const double vi = vt[i];
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j < w && j != t) d[j] += vi * V[i + (long long)j * ldv];
    }
    wave_sum_multi<NB>(d);
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < NB; ++j) red[wave][j] = d[j];
    }
    __syncthreads();
    if (tid < w && tid != t) {
      double s = V[t + (long long)tid * ldv];
      for (int q = 0; q < NWV; ++q) s += red[q][tid];
      sums[tid] = s;
    }
    __syncthreads();
    // T(0:t, t) = -tau T(0:t, 0:t) d(0:t); T(t, t) = tau
    if (tid < t) {
      double s = 0.0;
      for (int q = tid; q < t; ++q) s += Ts[tid][q] * sums[q];
      Ts[tid][t] = -tau * s;
    }
    if (tid == 0) Ts[t][t] = tau;
    // update columns j > t: A(t:h, j) -= tau d_j v
    const int nup = w - t - 1;
    if (nup > 0 && tau != 0.0) {
      for (long long e = tid; e < (long long)(h - t) * nup; e += QR_NT) {
        const int i = t + (int)(e % (h - t));
        const int j = t + 1 + (int)(e / (h - t));
        const double vi = (i == t) ? 1.0 : vt[i];
        V[i + (long long)j * ldv] -= tau * sums[j] * vi;
      }
    }
    __syncthreads();
  }

  // write R back (logical rows 0..w-1 = physical r1a..), zero the rest of the panel columns;
  // then clear V above its unit diagonal and store T.
  for (long long e = tid; e < (long long)h * w; e += QR_NT) {
    const int i = (int)(e % h), j = (int)(e / h);
    double val;
    if (i < j) val = V[i + (long long)j * ldv];
    else if (i == j) val = betas[j];
    else val = 0.0;
    M[qr_phys(i, h1, r1a, r2a) + (long long)(c0 + j) * ldm] = val;
  }
  __syncthreads();
  for (long long e = tid; e < (long long)w * w; e += QR_NT) {
    const int i = (int)(e % w), j = (int)(e / w);
    if (i < j) V[i + (long long)j * ldv] = 0.0;
  }
  for (int e = tid; e < NB * NB; e += QR_NT) {
    const int i = e % NB, j = e / NB;
    T[i + (long long)j * NB] = (i < w && j < w) ? Ts[i][j] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// host side

static void panel_segments(QRShape shape, int m, int n, int nb, int k, int* c0, int* w, int* r1a,
                           int* r1b, int* r2a, int* r2b) {
  *c0 = k * nb;
  *w = std::min(nb, n - *c0);
  if (shape == QRShape::General) {
    *r1a = *c0;
    *r1b = m;
    *r2a = *r2b = 0;
  } else {  // stacked [R; D], R and D n x n, m = 2n
    *r1a = *c0;
    *r1b = *c0 + *w;
    *r2a = n;
    *r2b = n + *c0 + *w;
  }
}

// Arena bytes that qr_work_alloc takes (allocation by allocation, with the
// arena's 256-byte alignment)
size_t qr_work_bytes(QRShape shape, int batch, int m, int n, int nb, int qcols) {
  auto al = [](size_t count) { return ((count * sizeof(double) + 255) / 256) * 256; };
  size_t t = 0;
  const int K = (n + nb - 1) / nb;
  constexpr int NBO = 128;
  const int hmax = (shape == QRShape::General) ? m : n + nb;
  const bool two = nb == 32 && n > nb && tsqr_panel_fits(hmax, nb);
  const int wcols = two ? NBO : nb;
  const int nblk = two ? (n + NBO - 1) / NBO : K;
  const long long ldv = (shape == QRShape::General) ? m : (n + wcols);
  const size_t sW = (size_t)wcols * std::max(n, qcols);
  const size_t ws_elems = (size_t)8 * batch * wcols * n;
  t += al((size_t)batch * nblk * ldv * wcols) + al((size_t)batch * K * nb * nb);
  t += 2 * al((size_t)batch * sW);
  if (nb == 32) t += tsqr_scratch_bytes(batch);
  t += al(ws_elems);
  if (two) {
    const int Ko = (n + NBO - 1) / NBO;
    t += al((size_t)batch * Ko * NBO * NBO) + al((size_t)batch * (NBO / nb) * nb * nb);
    t += al((size_t)batch * NBO * NBO);
    t += al((size_t)batch * ((hmax + PU_CH - 1) / PU_CH) * PU_W * PU_NC) + al(((size_t)batch + 1) / 2);
  }
  return t;
}

QRWork qr_work_alloc(Arena& ar, QRShape shape, int batch, int m, int n, int nb, int qcols) {
  QRWork wk;
  wk.nb = nb;
  wk.K = (n + nb - 1) / nb;
  wk.ar = &ar;
  // two-level blocking when every inner panel takes the TSQR path (tallest
  // panel: m rows for General, n + nb for Stacked) and there are several panels
  constexpr int NBO = 128;
  const int hmax = (shape == QRShape::General) ? m : n + nb;
  if (nb == 32 && n > nb && tsqr_panel_fits(hmax, nb)) {
    wk.nbo = NBO;
    wk.Ko = (n + NBO - 1) / NBO;
  }
  const int wcols = wk.nbo ? wk.nbo : nb;
  const int nblk = wk.nbo ? wk.Ko : wk.K;
  wk.ldv = (shape == QRShape::General) ? m : (n + wcols);
  wk.sV = (long long)nblk * wk.ldv * wcols;
  wk.sT = (long long)wk.K * nb * nb;
  wk.V = ar.dalloc((size_t)batch * wk.sV);
  wk.T = ar.dalloc((size_t)batch * wk.sT);
  wk.sW = (long long)wcols * std::max(n, qcols);
  wk.W = ar.dalloc((size_t)batch * wk.sW);
  wk.W2 = ar.dalloc((size_t)batch * wk.sW);
  if (nb == 32) wk.ts = tsqr_scratch_alloc(ar, batch);
  wk.ws_elems = (size_t)8 * batch * wcols * n;
  wk.ws = ar.dalloc(wk.ws_elems);
  if (wk.nbo) {
    wk.sTo = (long long)wk.Ko * NBO * NBO;
    wk.To = ar.dalloc((size_t)batch * wk.sTo);
    wk.sTin = (long long)(NBO / nb) * nb * nb;
    wk.Tin = ar.dalloc((size_t)batch * wk.sTin);
    wk.sG = (long long)NBO * NBO;
    wk.G = ar.dalloc((size_t)batch * wk.sG);
    // inner-panel updates: ceil(hmax / PU_CH) partials of 32 x 96 per problem
    const int nchunk = (hmax + PU_CH - 1) / PU_CH;
    wk.sPart = (long long)nchunk * 32 * 96;
    wk.pu_part = ar.dalloc((size_t)batch * wk.sPart);
    wk.pu_cnt = reinterpret_cast<unsigned*>(ar.dalloc(((size_t)batch + 1) / 2));
  }
  return wk;
}

// C <- (I - V T' V^T) C on the panel's row segments, columns [col0, col0 + nc);
// T' = T^T when transT (apply Q^T), T' = T otherwise (apply Q).
static void apply_block_reflector(int batch, double* M, long long ldm, long long sM, int col0,
                                  int nc, int r1a, int r1b, int r2a, int r2b, int w,
                                  const double* V, const double* V2, long long ldv, long long sV,
                                  const double* T, long long sT, int nbT, double* W, double* W2,
                                  long long sW, bool transT, double* ws, size_t ws_elems,
                                  hipStream_t s) {
  if (nc <= 0 || w <= 0) return;
  const int h1 = r1b - r1a, h2 = r2b - r2a;
  GemmBatch g;
  g.batch = batch;
  // W = V1^T C1 (+ V2^T C2)
  g.transA = 1; g.transB = 0;
  g.m = w; g.n = nc; g.k = h1;
  g.A = V; g.lda = ldv; g.sA = sV;
  g.B = M + r1a + (long long)col0 * ldm; g.ldb = ldm; g.sB = sM;
  g.C = W; g.ldc = w; g.sC = sW;
  g.alpha = 1.0; g.beta = 0.0;
  g.ws = ws; g.ws_elems = ws_elems;
  dgemm(g, s);
  if (h2 > 0) {
    g.k = h2;
    g.A = V2; g.B = M + r2a + (long long)col0 * ldm;
    g.beta = 1.0;
    dgemm(g, s);
  }
  // W2 = T' W
  GemmBatch t;
  t.batch = batch;
  t.transA = transT ? 1 : 0; t.transB = 0;
  t.m = w; t.n = nc; t.k = w;
  t.A = T; t.lda = nbT; t.sA = sT;
  t.B = W; t.ldb = w; t.sB = sW;
  t.C = W2; t.ldc = w; t.sC = sW;
  t.alpha = 1.0; t.beta = 0.0;
  dgemm(t, s);
  // C -= V W2
  GemmBatch u;
  u.batch = batch;
  u.transA = 0; u.transB = 0;
  u.m = h1; u.n = nc; u.k = w;
  u.A = V; u.lda = ldv; u.sA = sV;
  u.B = W2; u.ldb = w; u.sB = sW;
  u.C = M + r1a + (long long)col0 * ldm; u.ldc = ldm; u.sC = sM;
  u.alpha = -1.0; u.beta = 1.0;
  dgemm(u, s);
  if (h2 > 0) {
    u.m = h2;
    u.A = V2;
    u.C = M + r2a + (long long)col0 * ldm;
    dgemm(u, s);
  }
}


// ---------------------------------------------------------------------------
// Inner-panel update of the two-level factorisation in two kernels:
// C <- (I - V T V^T)^T C on the panel's logical rows (segment 1, then segment
// 2 of a Stacked panel) and the <= 96 columns left in the outer block.
//   pu_partial: each workgroup forms V_c^T C_c over PU_CH logical rows (FP64
//     MFMA, operands staged through LDS 64 rows at a time) and stores it; the
//     last workgroup of a problem to finish (counter) sums the partials in a
//     fixed order and writes W2 = T^T (V^T C) (32 x nc, ld 32).
//   pu_apply: C_r -= V_r W2 for 64-row tiles.

typedef double d4 __attribute__((ext_vector_type(4)));

// lane l, item v of the accumulator of a 16 x 16 block: row l % 16, column 4 v + l / 16
template <int KD, class FX, class FY>
__device__ __forceinline__ d4 pu_mfma(d4 acc, FX fx, FY fy, int ti, int tj) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < KD; kk += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fy(kk + lk, 16 * tj + lr), fx(16 * ti + lr, kk + lk),
                                               acc, 0, 0, 0);
  return acc;
}

__device__ __forceinline__ long long pu_mrow(int i, int h1, int r1a, int r2a) {
  return i < h1 ? r1a + i : r2a + (i - h1);
}
__device__ __forceinline__ long long pu_vrow(int i, int h1, int vr2) { return i < h1 ? i : vr2 + (i - h1); }

__global__ __launch_bounds__(256) void pu_partial_kernel(
    int h, int h1, int nc, const double* V, long long ldv, long long sV, int vr2, const double* M,
    long long ldm, long long sM, int r1a, int r2a, int col0, const double* T, int ldt, long long sT,
    double* part, long long sPart, double* W2, long long sW2, unsigned* cnt) {
  constexpr int NV = PU_SUB * PU_W / 256, NCL = PU_SUB * PU_NC / 256;  // staged values per thread
  __shared__ double Vs[PU_SUB][PU_W + 1];
  __shared__ double Cs[PU_SUB][PU_NC + 1];  // C rows while staging, then W (first 32 rows)
  __shared__ unsigned is_last;
  const int c = blockIdx.x, nchunk = gridDim.x;
  const long long b = blockIdx.y;
  V += b * sV;
  M += b * sM;
  T += b * sT;
  part += b * sPart;
  W2 += b * sW2;
  const int tid = threadIdx.x, wave = tid >> 6;
  const int ntj = (nc + 15) / 16, ntiles = 2 * ntj;  // 16 x 16 blocks of the 32 x nc product
  d4 acc[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
  // rows are staged PU_SUB at a time; the next rows are loaded into registers
  // while the current ones are multiplied
  double rv[NV], rc[NCL];
  auto load = [&](int r0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = tid + 256 * q, i = e % PU_SUB, j = e / PU_SUB;
      rv[q] = (r0 + i < h) ? V[pu_vrow(r0 + i, h1, vr2) + (long long)j * ldv] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NCL; ++q) {
      const int e = tid + 256 * q, i = e % PU_SUB, j = e / PU_SUB;
      rc[q] = (r0 + i < h && j < nc) ? M[pu_mrow(r0 + i, h1, r1a, r2a) + (long long)(col0 + j) * ldm] : 0.0;
    }
  };
  const int rbeg = c * PU_CH, rend = min(h, (c + 1) * PU_CH);
  load(rbeg);
  for (int r0 = rbeg; r0 < rend; r0 += PU_SUB) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int e = tid + 256 * q;
      Vs[e % PU_SUB][e / PU_SUB] = rv[q];
    }
#pragma unroll
    for (int q = 0; q < NCL; ++q) {
      const int e = tid + 256 * q;
      Cs[e % PU_SUB][e / PU_SUB] = rc[q];
    }
    __syncthreads();
    if (r0 + PU_SUB < rend) load(r0 + PU_SUB);
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int t = wave + 4 * u;
      if (t < ntiles)
        acc[u] = pu_mfma<PU_SUB>(acc[u], [&](int i, int k) { return Vs[k][i]; },
                                 [&](int k, int j) { return Cs[k][j]; }, t & 1, t >> 1);
    }
  }
  // this chunk's 32 x nc partial, row-major with row length 96
  double* pc = part + (long long)c * PU_W * PU_NC;
  const int lane = tid & 63;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int t = wave + 4 * u;
    if (t < ntiles) {
      const int row = 16 * (t & 1) + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) pc[row * PU_NC + 16 * (t >> 1) + 4 * v + (lane >> 4)] = acc[u][v];
    }
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) is_last = (atomicAdd(&cnt[b], 1u) == (unsigned)(nchunk - 1)) ? 1u : 0u;
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  // the last workgroup: W = sum of the partials in chunk order (all loads of
  // four chunks in flight at once), then W2 = T^T W
  constexpr int NE = PU_W * PU_NC / 256;
  double sacc[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) sacc[u] = 0.0;
  int q = 0;
  for (; q + 4 <= nchunk; q += 4) {
    double x[4][NE];
#pragma unroll
    for (int z = 0; z < 4; ++z)
#pragma unroll
      for (int u = 0; u < NE; ++u) x[z][u] = part[(long long)(q + z) * PU_W * PU_NC + tid + 256 * u];
#pragma unroll
    for (int z = 0; z < 4; ++z)
#pragma unroll
      for (int u = 0; u < NE; ++u) sacc[u] += x[z][u];
  }
  for (; q < nchunk; ++q) {
#pragma unroll
    for (int u = 0; u < NE; ++u) sacc[u] += part[(long long)q * PU_W * PU_NC + tid + 256 * u];
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + 256 * u;
    Cs[e / PU_NC][e % PU_NC] = sacc[u];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int t = wave + 4 * u;
    if (t < ntiles) {
      const d4 r = pu_mfma<PU_W>(d4{0.0, 0.0, 0.0, 0.0}, [&](int i, int k) { return T[k + (long long)i * ldt]; },
                                 [&](int k, int j) { return Cs[k][j]; }, t & 1, t >> 1);
      const int row = 16 * (t & 1) + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = 16 * (t >> 1) + 4 * v + (lane >> 4);
        if (col < nc) W2[row + (long long)col * PU_W] = r[v];
      }
    }
  }
  if (tid == 0) cnt[b] = 0u;
}

__global__ __launch_bounds__(256) void pu_apply_kernel(int h, int h1, int nc, const double* V,
                                                       long long ldv, long long sV, int vr2,
                                                       double* M, long long ldm, long long sM,
                                                       int r1a, int r2a, int col0, const double* W2,
                                                       long long sW2) {
  __shared__ double Ws[PU_W][PU_NC + 1];
  __shared__ double Vs[PU_RT][PU_W + 1];
  const int r0 = blockIdx.x * PU_RT;
  const long long b = blockIdx.y;
  V += b * sV;
  M += b * sM;
  W2 += b * sW2;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  {
    // all loads of a thread in flight at once, then the LDS stores
    constexpr int NW2 = PU_W * PU_NC / 256, NVL = PU_RT * PU_W / 256;
    double wv[NW2], vv[NVL];
#pragma unroll
    for (int q = 0; q < NW2; ++q) {
      const int e = tid + 256 * q, i = e % PU_W, j = e / PU_W;
      wv[q] = (j < nc) ? W2[i + (long long)j * PU_W] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NVL; ++q) {
      const int e = tid + 256 * q, i = e % PU_RT, j = e / PU_RT;
      vv[q] = (r0 + i < h) ? V[pu_vrow(r0 + i, h1, vr2) + (long long)j * ldv] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NW2; ++q) {
      const int e = tid + 256 * q;
      Ws[e % PU_W][e / PU_W] = wv[q];
    }
#pragma unroll
    for (int q = 0; q < NVL; ++q) {
      const int e = tid + 256 * q;
      Vs[e % PU_RT][e / PU_RT] = vv[q];
    }
  }
  __syncthreads();
  const int ntj = (nc + 15) / 16;
  // wave w owns the 16-row tile w and every 16-column tile: all products,
  // then all old values (loaded together), then the stores
  constexpr int NTJ = PU_NC / 16;
  const int row = r0 + 16 * wave + (lane & 15);
  const bool rok = row < h;
  const long long mr = rok ? pu_mrow(row, h1, r1a, r2a) : 0;
  d4 r[NTJ];
#pragma unroll
  for (int u = 0; u < NTJ; ++u)
    if (u < ntj)
      r[u] = pu_mfma<PU_W>(d4{0.0, 0.0, 0.0, 0.0}, [&](int i, int k) { return Vs[i][k]; },
                           [&](int k, int j) { return Ws[k][j]; }, wave, u);
  double o[NTJ][4];
#pragma unroll
  for (int u = 0; u < NTJ; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = 16 * u + 4 * v + (lane >> 4);
      o[u][v] = (rok && u < ntj && col < nc) ? M[mr + (long long)(col0 + col) * ldm] : 0.0;
    }
#pragma unroll
  for (int u = 0; u < NTJ; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (u < ntj) o[u][v] -= r[u][v];
#pragma unroll
  for (int u = 0; u < NTJ; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = 16 * u + 4 * v + (lane >> 4);
      if (rok && u < ntj && col < nc) M[mr + (long long)(col0 + col) * ldm] = o[u][v];
    }
}

// One workgroup per problem: the compact-WY factor T (w x w, w <= 128) of an
// outer block from the factors T_k of its 32-wide inner panels and the Gram
// matrix G = V^T V of the block's vectors, one column block at a time:
// T(0:c, c:c+32) = -T(0:c, 0:c) (G(0:c, c:c+32) T_jj), c = 32 j (the factor
// of H_0 ... H_j from those of H_0 ... H_{j-1} and H_j).  A panel step with
// tau = 0 (H = I) keeps its zero row and column of T_k, and so of T.
__global__ __launch_bounds__(256) void ut_merge_kernel(int w, const double* __restrict__ G,
                                                       long long ldg, long long sG,
                                                       const double* __restrict__ Tin,
                                                       long long sTin, double* T, long long ldt,
                                                       long long sT) {
  constexpr int B = PU_W, BB = PU_W * PU_W;  // inner panel width and factor size
  static_assert(4 * B == 128, "index maps below assume 128 columns");
  __shared__ double Tl[3 * B][4 * B + 1];    // rows 0..95 of T
  __shared__ double Xs[3 * B][B + 1];        // G block, then X
  __shared__ double Tj[B][B + 1];            // T_jj
  const long long b = blockIdx.x;
  G += b * sG;
  Tin += b * sTin;
  T += b * sT;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int npan = (w + B - 1) / B;
  // every global input is loaded once, all loads of a thread in flight at
  // once: the four panel factors (element e = tid + 256 q of the 4 x 32 x 32
  // array) and the Gram region G(0:96, 32:128) that the merges read (element
  // e: row e % 96, column 32 + e / 96; zero beyond w)
  constexpr int NT_ = 4 * BB / 256, NG = 3 * B * 3 * B / 256;
  double tv[NT_], gv[NG];
#pragma unroll
  for (int q = 0; q < NT_; ++q) {
    const int e = tid + 256 * q;
    tv[q] = (e / BB < npan) ? Tin[e] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const int e = tid + 256 * q, i = e % (3 * B), c = B + e / (3 * B);
    gv[q] = (c < w && i < c) ? G[i + (long long)c * ldg] : 0.0;
  }
  for (int e = tid; e < 3 * B * 4 * B; e += 256) Tl[e >> 7][e & 127] = 0.0;  // 4 B = 128 columns
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NT_; ++q) {
    const int e = tid + 256 * q, blk = e / BB, i = e % B, j = (e % BB) / B;
    if (blk < 3) Tl[B * blk + i][B * blk + j] = tv[q];
  }
  __syncthreads();
  for (int jb = 1; jb < npan; ++jb) {
    const int c0 = B * jb;
    const int ntile = (c0 / 16) * 2;
    // stage G(0:c0, c0:c0+32) and T_jj from the registers
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      const int e = tid + 256 * q, i = e % (3 * B), c = B + e / (3 * B);
      if (c >= c0 && c < c0 + B && i < c0) Xs[i][c - c0] = gv[q];
    }
#pragma unroll
    for (int q = 0; q < NT_; ++q) {
      const int e = tid + 256 * q;
      if (e / BB == jb) Tj[e % B][(e % BB) / B] = tv[q];
    }
    __syncthreads();
    // X = G(0:c0, c0:c0+32) T_jj, in registers, then over the staged G block
    d4 x[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int t = wave + 4 * u;
      if (t < ntile)
        x[u] = pu_mfma<B>(d4{0.0, 0.0, 0.0, 0.0}, [&](int i, int k) { return Xs[i][k]; },
                          [&](int k, int j) { return Tj[k][j]; }, t >> 1, t & 1);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int t = wave + 4 * u;
      if (t < ntile) {
        const int ti = t >> 1, tj = t & 1;
#pragma unroll
        for (int v = 0; v < 4; ++v) Xs[16 * ti + (lane & 15)][16 * tj + 4 * v + (lane >> 4)] = x[u][v];
      }
    }
    __syncthreads();
    // T(0:c0, c0:c0+32) = -T(0:c0, 0:c0) X
    for (int t = wave; t < ntile; t += 4) {
      const int ti = t >> 1, tj = t & 1;
      auto fx = [&](int i, int k) { return Tl[i][k]; };
      auto fy = [&](int k, int j) { return Xs[k][j]; };
      d4 r;
      if (jb == 1) r = pu_mfma<B>(d4{0.0, 0.0, 0.0, 0.0}, fx, fy, ti, tj);
      else if (jb == 2) r = pu_mfma<2 * B>(d4{0.0, 0.0, 0.0, 0.0}, fx, fy, ti, tj);
      else r = pu_mfma<3 * B>(d4{0.0, 0.0, 0.0, 0.0}, fx, fy, ti, tj);
#pragma unroll
      for (int v = 0; v < 4; ++v) Tl[16 * ti + (lane & 15)][c0 + 16 * tj + 4 * v + (lane >> 4)] = -r[v];
    }
    __syncthreads();
  }
  // rows 96.. of T: T_33 on the diagonal block (Xs is free: stage it there)
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NT_; ++q) {
    const int e = tid + 256 * q;
    if (e / BB == 3) Xs[e % B][(e % BB) / B] = tv[q];
  }
  __syncthreads();
  for (int e = tid; e < 4 * B * 4 * B; e += 256) {
    const int i = e & (4 * B - 1), j = e >> 7;
    if (i < w && j < w) {
      double v;
      if (i < 3 * B) v = Tl[i][j];
      else v = (j >= 3 * B) ? Xs[i - 3 * B][j - 3 * B] : 0.0;
      T[i + (long long)j * ldt] = v;
    }
  }
}

__global__ void zero_u32_kernel(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// the two kernels above for one inner panel (w <= 32, nc <= 96), T = T_k (ld nb)
static void inner_update(int batch, int h1, int h, int nc, const double* V, long long ldv,
                         long long sV, int vr2, double* M, long long ldm, long long sM, int r1a,
                         int r2a, int col0, const double* T, int ldt, long long sT, double* W2,
                         long long sW2, const QRWork& wk, hipStream_t s) {
  if (nc <= 0) return;
  if (nc > PU_NC) throw ArgError("inner_update: too many columns");
  const int nchunk = (h + PU_CH - 1) / PU_CH;
  if ((long long)nchunk * PU_W * PU_NC > wk.sPart) throw ArgError("inner_update: panel too tall");
  {
    ProfScope prof("qr_inner_w", s, batch * 2.0 * PU_W * nc * (double)h + batch * 2.0 * PU_W * PU_W * nc,
                   batch * 8.0 * (double)h * (PU_W + nc));
    hipLaunchKernelGGL(pu_partial_kernel, dim3(nchunk, batch), dim3(256), 0, s, h, h1, nc, V, ldv, sV,
                       vr2, M, ldm, sM, r1a, r2a, col0, T, ldt, sT, wk.pu_part, wk.sPart, W2, sW2,
                       wk.pu_cnt);
    ZCSD_CHECK_LAUNCH();
  }
  {
    ProfScope prof("qr_inner_apply", s, batch * 2.0 * PU_W * nc * (double)h,
                   batch * 8.0 * (double)h * (PU_W + 2.0 * nc));
    hipLaunchKernelGGL(pu_apply_kernel, dim3((h + PU_RT - 1) / PU_RT, batch), dim3(256), 0, s, h,
                       h1, nc, V, ldv, sV, vr2, M, ldm, sM, r1a, r2a, col0, W2, sW2);
    ZCSD_CHECK_LAUNCH();
  }
}

// Two-level blocked factorisation: inside an outer block of nbo columns the
// inner panels are factored and applied to the rest of the block only; the
// outer block's compact-WY factor follows from the inner panels' factors and
// the Gram matrix of its vectors (ut_merge_kernel), and the trailing
// columns get one update with inner dimension nbo, which reads and writes the
// trailing matrix nbo / nb times less often than panel-by-panel updates.
// In the outer block's V, the first segment's rows come first and the second
// segment (Stacked) starts at row wo, so both segments are contiguous.
static void geqrf_two_level(int batch, QRShape shape, int m, int n, double* M, long long ldm,
                            long long sM, QRWork& wk, hipStream_t s) {
  const int nb = wk.nb, NBO = wk.nbo;
  // the inner-update counters start at zero (each use leaves them at zero)
  hipLaunchKernelGGL(zero_u32_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, wk.pu_cnt, batch);
  ZCSD_CHECK_LAUNCH();
  for (int O = 0; O < wk.Ko; ++O) {
    const int co = O * NBO, wo = std::min(NBO, n - co);
    double* VO = wk.V + (long long)O * wk.ldv * NBO;
    double* TO = wk.To + (long long)O * NBO * NBO;
    const bool gen = shape == QRShape::General;
    const int orows = gen ? (m - co) : (2 * wo + co);  // rows of VO in use
    set_identity(batch, (int)wk.ldv, NBO, 0.0, VO, wk.ldv, wk.sV, s);
    const int npan = (wo + nb - 1) / nb;
    for (int kk = 0; kk < npan; ++kk) {
      const int c0 = co + kk * nb, w = std::min(nb, n - c0);
      int r1a, r1b, r2a, r2b;
      if (gen) {
        r1a = c0; r1b = m; r2a = r2b = 0;
      } else {
        r1a = c0; r1b = c0 + w; r2a = n; r2b = n + c0 + w;
      }
      const int off = c0 - co;
      double* V1 = VO + off + (long long)off * wk.ldv;
      double* V2 = VO + wo + (long long)off * wk.ldv;
      const int vr2 = gen ? -1 : (wo - off);
      double* Tk = wk.Tin + (long long)kk * nb * nb;
      tsqr_panel(batch, M, ldm, sM, c0, w, r1a, r1b, r2a, r2b, V1, wk.ldv, wk.sV, vr2, Tk, wk.sTin,
                 wk.ts, s);
      const int col0 = c0 + w;
      // V2 - V1 = wo - off rows: segment 2 of the logical rows starts there
      inner_update(batch, r1b - r1a, (r1b - r1a) + (r2b - r2a), co + wo - col0, V1, wk.ldv, wk.sV,
                   gen ? 0 : (wo - off), M, ldm, sM, r1a, r2a, col0, Tk, nb, wk.sTin, wk.W2, wk.sW,
                   wk, s);
    }
    // outer compact-WY factor from the inner factors and G = VO^T VO (always FP64)
    {
      GemmFp64Scope fp64;
      GemmBatch g;
      g.batch = batch;
      g.transA = 1;
      g.m = wo; g.n = wo; g.k = orows;
      g.A = VO; g.lda = wk.ldv; g.sA = wk.sV;
      g.B = VO; g.ldb = wk.ldv; g.sB = wk.sV;
      g.C = wk.G; g.ldc = NBO; g.sC = wk.sG;
      g.ws = wk.ws; g.ws_elems = wk.ws_elems;
      g.sym_upper = true;  // the merge reads only blocks above the diagonal
      dgemm(g, s);
      if (nb != PU_W || NBO > 4 * PU_W) throw ArgError("geqrf: outer block layout");
      hipLaunchKernelGGL(ut_merge_kernel, dim3(batch), dim3(256), 0, s, wo, wk.G, (long long)NBO,
                         wk.sG, wk.Tin, wk.sTin, TO, (long long)NBO, wk.sTo);
      ZCSD_CHECK_LAUNCH();
    }
    const int col0 = co + wo;
    if (col0 < n) {
      int r1a, r1b, r2a, r2b;
      if (gen) {
        r1a = co; r1b = m; r2a = r2b = 0;
      } else {
        r1a = co; r1b = co + wo; r2a = n; r2b = n + co + wo;
      }
      apply_block_reflector(batch, M, ldm, sM, col0, n - col0, r1a, r1b, r2a, r2b, wo, VO, VO + wo,
                            wk.ldv, wk.sV, TO, wk.sTo, NBO, wk.W, wk.W2, wk.sW, /*transT=*/true,
                            wk.ws, wk.ws_elems, s);
    }
  }
}

void geqrf_batched(int batch, QRShape shape, int m, int n, double* M, long long ldm, long long sM,
                   QRWork& wk, hipStream_t s) {
  if (batch <= 0 || n <= 0) return;
  if (wk.nbo) {
    geqrf_two_level(batch, shape, m, n, M, ldm, sM, wk, s);
    return;
  }
  const int nb = wk.nb;
  for (int k = 0; k < wk.K; ++k) {
    int c0, w, r1a, r1b, r2a, r2b;
    panel_segments(shape, m, n, nb, k, &c0, &w, &r1a, &r1b, &r2a, &r2b);
    double* Vk = wk.V + (long long)k * wk.ldv * nb;
    double* Tk = wk.T + (long long)k * nb * nb;
    const double hh = (double)(r1b - r1a) + (r2b - r2a);
    // a panel is either the three TSQR kernels or the one-workgroup kernel
    if (nb == 32 && wk.ts.Rstack && tsqr_panel_fits((int)hh, w)) {
      tsqr_panel(batch, M, ldm, sM, c0, w, r1a, r1b, r2a, r2b, Vk, wk.ldv, wk.sV, -1, Tk, wk.sT,
                 wk.ts, s);
    } else {
      ProfScope prof("qr_panel", s, batch * 2.0 * hh * w * w, batch * 8.0 * 2.0 * hh * w);
      if (nb == 32)
        hipLaunchKernelGGL(qr_panel_kernel<32>, dim3(batch), dim3(QR_NT), 0, s, M, ldm, sM, c0, w,
                           r1a, r1b, r2a, r2b, Vk, wk.ldv, wk.sV, Tk, wk.sT);
      else if (nb == 16)
        hipLaunchKernelGGL(qr_panel_kernel<16>, dim3(batch), dim3(QR_NT), 0, s, M, ldm, sM, c0, w,
                           r1a, r1b, r2a, r2b, Vk, wk.ldv, wk.sV, Tk, wk.sT);
      else
        throw ArgError("geqrf: unsupported panel width");
      ZCSD_CHECK_LAUNCH();
    }
    const int col0 = c0 + w;
    const int h1 = r1b - r1a;
    apply_block_reflector(batch, M, ldm, sM, col0, n - col0, r1a, r1b, r2a, r2b, w, Vk, Vk + h1,
                          wk.ldv, wk.sV, Tk, wk.sT, nb, wk.W, wk.W2, wk.sW, /*transT=*/true, wk.ws,
                          wk.ws_elems, s);
  }
}

void orgqr_batched(int batch, QRShape shape, int m, int n, double* Q, long long ldq, long long sQ,
                   const double* d_scale, const QRWork& wk, hipStream_t s, int qcols) {
  if (batch <= 0 || n <= 0) return;
  // Q has nq columns: the n reflectors applied to the first nq columns of I_m
  const int nq = std::max(n, qcols);
  if (nq > n && (shape != QRShape::General || nq > m))
    throw ArgError("orgqr: more columns than reflectors needs a General shape and nq <= m");
  if (wk.sW < (long long)(wk.nbo ? wk.nbo : wk.nb) * nq)
    throw ArgError("orgqr: workspace sized for fewer columns of Q");
  set_identity_scaled(batch, m, nq, d_scale, 1.0, Q, ldq, sQ, s);
  if (wk.nbo) {
    const int NBO = wk.nbo;
    for (int O = wk.Ko - 1; O >= 0; --O) {
      const int co = O * NBO, wo = std::min(NBO, n - co);
      const double* VO = wk.V + (long long)O * wk.ldv * NBO;
      const double* TO = wk.To + (long long)O * NBO * NBO;
      int r1a, r1b, r2a, r2b;
      if (shape == QRShape::General) {
        r1a = co; r1b = m; r2a = r2b = 0;
      } else {
        r1a = co; r1b = co + wo; r2a = n; r2b = n + co + wo;
      }
      apply_block_reflector(batch, Q, ldq, sQ, co, nq - co, r1a, r1b, r2a, r2b, wo, VO, VO + wo,
                            wk.ldv, wk.sV, TO, wk.sTo, NBO, wk.W, wk.W2, wk.sW, /*transT=*/false,
                            wk.ws, wk.ws_elems, s);
    }
    return;
  }
  const int nb = wk.nb;
  for (int k = wk.K - 1; k >= 0; --k) {
    int c0, w, r1a, r1b, r2a, r2b;
    panel_segments(shape, m, n, nb, k, &c0, &w, &r1a, &r1b, &r2a, &r2b);
    const double* Vk = wk.V + (long long)k * wk.ldv * nb;
    const double* Tk = wk.T + (long long)k * nb * nb;
    const int h1 = r1b - r1a;
    apply_block_reflector(batch, Q, ldq, sQ, c0, nq - c0, r1a, r1b, r2a, r2b, w, Vk, Vk + h1, wk.ldv,
                          wk.sV, Tk, wk.sT, nb, wk.W, wk.W2, wk.sW, /*transT=*/false, wk.ws,
                          wk.ws_elems, s);
  }
}

}  // namespace zcsd
