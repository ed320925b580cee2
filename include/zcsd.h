/*
 * zcsd.h -- C ABI of libzcsd, an MI355X (gfx950) implementation of the CS
 * decomposition of Gawlik, Nakatsukasa & Sutton, "A Backward Stable Algorithm
 * for Computing the CS Decomposition via the Polar Decomposition"
 * (arXiv 1804.09002): Zolo-csd = two Zolotarev polar decompositions (Zolo-pd,
 * Sec. 5), the Hermitian matrix B = H2 - H1 + mu (I - A^T A) (Algorithm 1)
 * and a Zolotarev spectral divide-and-conquer eigendecomposition of B
 * (Zolo-eig, Sec. 5), assembled into U1, U2, V1 and the angles theta.
 *
 * Conventions for every entry point
 *  - Matrices are real FP64, column-major, with a leading dimension ld >= rows
 *    (zcsd_zcsd: interleaved complex FP64, ld counted in complex elements).
 *  - Pointers named d_* are device pointers (HIP memory on the handle's device);
 *    h_* are host pointers.  The caller owns all input and output buffers.
 *  - Work is enqueued on the handle's stream.  Entry points that need host
 *    decisions (rank, Zolotarev degree, divide-and-conquer split sizes)
 *    synchronise that stream internally; when an entry point returns
 *    ZCSD_OK its outputs are complete and the info struct is filled.
 *  - Inputs are not modified; outputs must not alias inputs.
 *  - Argument errors return ZCSD_EINVAL before any work is enqueued.
 *    HIP runtime failures return ZCSD_EHIP; allocation failures ZCSD_ENOMEM.
 *    Numerical conditions are reported through the status and zcsd_info.
 *  - A handle is not thread-safe; use one handle per host thread.
 *  - Workspace: the entry points take no caller workspace.  Each handle owns
 *    one device arena that grows to the largest size a call has needed and is
 *    reused by later calls (no allocation inside a call once it has grown);
 *    zcsd_workspace_size reports its size for a square CSD beforehand.  The
 *    amount a call needs depends on host decisions made during the call
 *    (Zolotarev degree, split sizes of Zolo-eig, size classes of a batch), so
 *    one bound per call would have to be the worst case of all of them.
 *    zcsd_dcsd_backward_noalloc is the one entry point that allocates nothing;
 *    zcsd_dcsd_batched_small, whose small problems need no host decision,
 *    takes a caller-owned workspace sized by zcsd_small_batch_prepare.
 */
#ifndef ZCSD_H
#define ZCSD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ZCSD_OK = 0,
  ZCSD_EINVAL = 1,   /* bad argument (size, leading dimension, NULL pointer, NaN/Inf input) */
  ZCSD_ENOTISO = 2,  /* input is far from a partial isometry: |‖A‖_F^2 - rank| too large (Sec. 2.1) */
  ZCSD_ENOCONV = 3,  /* Zolo-pd did not reach 1 - l_2 <= tol, or a split of Zolo-eig failed */
  ZCSD_EREPAIR = 4,  /* Algorithm 2 repair rejected (‖R~ - R‖_F > 100 n u ‖R‖_F, Sec. 5.1) */
  ZCSD_EHIP = 5,     /* HIP runtime error */
  ZCSD_ENOMEM = 6    /* device allocation failed */
} zcsd_status;

/* ZCSD_MIXED_FP32 (not in the paper): the products of the Cholesky-form
 * iteration of both polar decompositions and every product of Zolo-eig run on
 * the FP32 matrix cores (operands rounded to FP32, FP32 accumulation, FP64
 * storage); the QR-form first iteration of the polars (ill-conditioned input),
 * B and the assembly stay FP64, and the polar factors and V1 each get one FP64
 * Newton-Schulz step; the Zolotarev degree is chosen as in the FP64 mode.
 * Products take the FP32 instructions where they did not measure slower than
 * FP64 (dense, untransposed second operand); transposed and triangular ones
 * stay FP64.  The results meet a stated tolerance of 1e-5 instead of the
 * FP64 mode's: backward error, orthogonality of U1, U2, V1 and angles carry
 * the FP32 products' error (measured 2-4e-6, 1e-10 and 1e-7 at n = 1024 and
 * 4096).  There is no FP64 fallback; info->lowp_products counts the FP32
 * products of the call.  Accepted by zcsd_dcsd, zcsd_dcsd_mn and
 * zcsd_dcsd2x2; zcsd_dcsd_batched is FP64 only. */
typedef enum { ZCSD_FP64 = 0, ZCSD_MIXED_FP32 = 1 } zcsd_precision;

typedef enum {
  ZCSD_RANK_AUTO = 0,      /* Remark (vi): rank = round(‖A‖_F^2); deficient iff rank < n */
  ZCSD_RANK_FULL = 1,      /* Algorithm 1 with mu = 0 */
  ZCSD_RANK_DEFICIENT = 2  /* Algorithm 3 with mu = opts.mu */
} zcsd_rank_mode;

/* Options.  zcsd_default_opts() fills the paper's values. */
typedef struct {
  zcsd_precision prec;     /* ZCSD_FP64 (default) or ZCSD_MIXED_FP32 (above) */
  zcsd_rank_mode rank_mode;
  double eps;              /* floor of the Zolo-pd interval [eps, 1]; 1e-15 (Sec. 5.1) */
  double mu;               /* shift of the null space in B; 2 (Algorithm 3) */
  double tol;              /* Zolo-pd target 1 - l_2 <= tol; 2^-53 */
  int r_override;          /* 0 = choose r from the l estimate; 1..8 forces r */
  double ell_override;     /* 0 = estimate l = sigma_min lower bound; > 0 forces l */
  int n_leaf;              /* Zolo-eig blocks of at most this size go to Jacobi (<= 64) */
  int postprocess;         /* 0, 1: C_ii = v_i^T H1 v_i, S_ii = v_i^T H2 v_i (Algorithm 1),
                              theta = atan2(S_ii, C_ii), C = cos, S = sin (Remark (iii));
                              2: theta_i solves sin(theta) - cos(theta) = Lambda_ii, the
                              cheaper and less accurate alternative of Remark (iv) (no
                              H_i V products); 1 is the default */
} zcsd_opts;

/* Diagnostics filled by zcsd_dcsd / zcsd_dzolo_pd / zcsd_dsyev_zolo. */
typedef struct {
  int rank;                /* numerical rank used (columns of U1, U2, V1 that are valid) */
  int r_used[2];           /* Zolotarev terms per iteration of the two polars (same r both steps) */
  double ell[2];           /* lower bounds l_0 used for the two polars */
  double zolo_resid;       /* 1 - l_2 of the coefficient sequence actually used */
  int eig_levels;          /* divide-and-conquer levels of Zolo-eig */
  int eig_splits;          /* number of successful splits */
  int eig_max_r;           /* largest Zolotarev degree used inside Zolo-eig */
  double eig_offblock;     /* max over splits of ‖V-^T B V+‖_F / ‖B‖_F (0 if not measured) */
  double eig_coupling;     /* max over splits of ‖X‖_F, the eigenspace-basis coupling that the
                              subspace-iteration step of each split removes */
  int eig_full_refinements; /* splits whose step needed a second QR (‖X‖_F > 2^-27) */
  int lowp_products;       /* products run on the FP32 matrix cores during the call (mixed
                              mode; 0 in the FP64 mode) */
  int repair;              /* 1 if Algorithm 2 (Sec. 5.1) replaced W_i = Q_i Q~_i^T (full rank:
                              when the sigma_min estimate reached eps; rank deficient: always
                              tried, kept when it passes the check) */
  double repair_resid;     /* its max_i ‖R~_i - R_i‖_F / ‖R_i‖_F (accepted below 100 n u) */
  double time_ms[4];       /* polar, B, eig, assembly wall time (ms), measured with stream syncs */
} zcsd_info;

typedef struct zcsd_handle_s zcsd_handle;

/* Create a handle on HIP device `device`; it owns a workspace arena and a stream
 * (the null stream until zcsd_set_stream is called).  Returns ZCSD_EHIP if the
 * device cannot be set. */
zcsd_status zcsd_create(zcsd_handle** handle, int device);
zcsd_status zcsd_destroy(zcsd_handle* handle);
/* Work is enqueued on `stream` (a hipStream_t passed as void*). */
zcsd_status zcsd_set_stream(zcsd_handle* handle, void* stream);
void zcsd_default_opts(zcsd_opts* opts);
const char* zcsd_status_string(zcsd_status s);
/* Tuning, per handle (mostly of the batched path, zcsd_dcsd_batched); not in the
 * paper.  The problems of a batch are grouped into size classes padded to
 * the next multiple of a step (ZCSD_TUNE_CLASS_STEP_SMALL for n <= 64,
 * default 8; _MID for 64 < n <= 256, default 16; _LARGE beyond, default 64),
 * and the groups run on ZCSD_TUNE_BATCHED_WORKERS concurrent host threads,
 * each with its own stream and workspace (default 4).  Smaller steps pad less
 * but make more groups; more workers overlap more latency-bound chains but
 * hold more workspace and compete for the device.  The defaults are the best
 * measured on 2048 problems with n log-uniform in [8, 256];
 * paper_1804_09002_amd/autotune.py measures the settings for another
 * workload.  Full-rank problems with n <= ZCSD_TUNE_ONE_WORKGROUP_MAX_N
 * (default 56, at most 64, 0 = none) skip the classes: each runs as a whole
 * CSD inside one workgroup, all of them in persistent launches by tier of
 * size (n <= 16: eight workgroups per compute unit; n <= 32: four; n <= 48:
 * two; n <= 64: one) that run beside the class groups (the same Algorithm 1 with
 * Zolo-pd; Zolo-eig of a block of at most 64 is its Jacobi leaf solve),
 * unless r_override, ell_override or n_leaf < n asks for the class path.
 * ZCSD_TUNE_GEMM_TILE128_MIN applies to every call of the handle: a matrix
 * product with at least that many 128 x 128 output tiles (over its batch)
 * uses the 128 x 128 tiling, the others 64 x 64 tiles (default 512, two per
 * compute unit); paper_1804_09002_amd/autotune.py measures it per problem
 * size and precision.  zcsd_set_tuning returns ZCSD_EINVAL for an
 * unknown key, workers outside [1, 16], a step outside [1, 256], a
 * one-workgroup limit outside [0, 64] or a tile threshold outside
 * [1, 2^24]; it takes effect on the next call of the handle. */
typedef enum {
  ZCSD_TUNE_BATCHED_WORKERS = 0,
  ZCSD_TUNE_CLASS_STEP_SMALL = 1,
  ZCSD_TUNE_CLASS_STEP_MID = 2,
  ZCSD_TUNE_CLASS_STEP_LARGE = 3,
  ZCSD_TUNE_ONE_WORKGROUP_MAX_N = 4,
  ZCSD_TUNE_GEMM_TILE128_MIN = 5
} zcsd_tune_key;
zcsd_status zcsd_set_tuning(zcsd_handle* handle, int key, int value);
zcsd_status zcsd_get_tuning(zcsd_handle* handle, int key, int* value);

/* sizeof(zcsd_opts) and sizeof(zcsd_info) as this library was built: a
 * binding that lays the structs out itself checks them before any call that
 * reads or writes one (a mismatch would make the library write past the
 * caller's struct). */
size_t zcsd_sizeof_opts(void);
size_t zcsd_sizeof_info(void);

/*
 * CS decomposition of A = [A1; A2], A1, A2 n x n (Sec. 1; Theorem 2.1 for a
 * rank-deficient partial isometry).  Algorithm 1, or Algorithm 3 when the
 * rank is (detected or forced) below n:
 *    A1 = U1 diag(cos theta) V1^T,  A2 = U2 diag(sin theta) V1^T,
 *    0 <= theta_1 <= ... <= theta_r <= pi/2 (Sec. 1), r = info->rank.
 * Outputs: d_U1, d_U2, d_V1 are n x n (ld >= n); only their first r columns
 * and the first r entries of d_theta (length n) are valid (economical CSD,
 * Remark (vii)); the rest are zero.  d_W1, d_W2 (optional, may be NULL)
 * receive the polar factors W_i (n x n, ld n) used by the backward pass.
 * opts may be NULL (defaults); info may be NULL.
 */
zcsd_status zcsd_dcsd(zcsd_handle* handle, int n,
                      const double* d_A1, int lda1, const double* d_A2, int lda2,
                      double* d_U1, int ldu1, double* d_U2, int ldu2,
                      double* d_V1, int ldv1, double* d_theta,
                      double* d_W1, double* d_W2,
                      const zcsd_opts* opts, zcsd_info* info);

/*
 * Device bytes the handle's arena holds for zcsd_dcsd / zcsd_dcsd2x2 at size n
 * (the polar batch of two n x n problems with up to eight Zolotarev terms,
 * the Zolo-eig levels of Sec. 5 and the assembly buffers; 28.2 GB at
 * n = 4096).  A host computation: nothing is enqueued or allocated, and
 * `handle` may be NULL.  Errors: ZCSD_EINVAL for n < 1, a NULL `bytes` or
 * out-of-range opts.
 */
zcsd_status zcsd_workspace_size(zcsd_handle* handle, int n, const zcsd_opts* opts, size_t* bytes);

/*
 * CS decomposition with rectangular blocks, A1 m1 x n and A2 m2 x n with
 * m1, m2 >= n (Algorithm 1 / Algorithm 3 as stated for m1 + m2 rows, Sec. 2
 * and Sec. 3): A1 = U1 diag(cos theta) V1^T, A2 = U2 diag(sin theta) V1^T with
 * U1 (m1 x n), U2 (m2 x n) and V1 (n x n) of orthonormal columns.  The blocks
 * are reduced by Householder QRs A_i = Q_i R_i: [R1; R2] is a 2n x n partial
 * isometry of the same rank and angles, polar(A_i) = Q_i polar(R_i), so the
 * square path runs on [R1; R2] and U_i = Q_i U_i'.  Column-major device
 * memory owned by the caller: d_A1 (ld >= m1), d_A2 (ld >= m2) are read
 * only; d_U1 (ld >= m1), d_U2 (ld >= m2), d_V1 (ld >= n) and d_theta
 * (length n) are written, with only the first info->rank columns / entries
 * valid (the rest zero).  opts may be NULL (defaults); info may be NULL.
 * Errors: ZCSD_EINVAL for m1 < n, m2 < n, n < 1, NULL pointers or short
 * leading dimensions (nothing enqueued); otherwise as zcsd_dcsd.  Returns
 * after the stream has finished the call.
 */
zcsd_status zcsd_dcsd_mn(zcsd_handle* handle, int m1, int m2, int n,
                         const double* d_A1, int lda1, const double* d_A2, int lda2,
                         double* d_U1, int ldu1, double* d_U2, int ldu2,
                         double* d_V1, int ldv1, double* d_theta,
                         const zcsd_opts* opts, zcsd_info* info);

/*
 * CS decomposition of a complex partial isometry A = [A1; A2], A1, A2 in
 * C^{n x n} (the setting of Sec. 1 and Theorem 2.1):
 *    A1 = U1 diag(cos theta) V1^*,  A2 = U2 diag(sin theta) V1^*,
 * U1, U2, V1 with orthonormal (complex) columns, theta ascending in
 * [0, pi/2].  Computed through the real embedding X + iY -> [X -Y; Y X]:
 * Algorithm 1 / 3 on the 2n x 2n real blocks, whose angles are those of A
 * twice; the complex columns are read from one real column of each pair,
 * repeated complex angles get a complex-orthonormal basis of their cluster,
 * Newton-Schulz steps on the embedded V1 (the same right factor on U1 and
 * U2) make the columns complex-orthonormal, U1 and U2 then get correction
 * steps of their own that change each column only by better-determined ones
 * (larger cos theta for U1, sin theta for U2), columns that A leaves
 * undetermined (cos or sin below 2^-46) are completed orthonormally, and the
 * angles are recomputed from the final factors.
 * Memory: column-major device arrays of interleaved complex doubles
 * (re, im), as std::complex<double> / hipDoubleComplex; leading dimensions
 * count complex elements (>= n).  d_A1, d_A2 are read only; d_U1, d_U2,
 * d_V1 (n x n) and d_theta (n reals) are written, with only the first
 * info->rank columns / entries valid (the rest zero).  opts may be NULL;
 * only prec = ZCSD_FP64 is accepted.  info may be NULL; it reports the rank
 * and whether Algorithm 2 replaced a polar factor.  Errors: ZCSD_EINVAL for
 * n outside [1, 32767], NULL pointers, short leading dimensions or another
 * precision;
 * ZCSD_ENOCONV as zcsd_dcsd, or when a real angle has no partner within the
 * pairing gap; ZCSD_ENOMEM when the workspace (11 (2n)^2 doubles plus what
 * zcsd_workspace_size reports for the real path at size 2n) cannot be
 * allocated.  Returns after the stream has finished the call.
 */
zcsd_status zcsd_zcsd(zcsd_handle* handle, int n,
                      const double* d_A1, int lda1, const double* d_A2, int lda2,
                      double* d_U1, int ldu1, double* d_U2, int ldu2,
                      double* d_V1, int ldv1, double* d_theta,
                      const zcsd_opts* opts, zcsd_info* info);

/*
 * zcsd_zcsd with rectangular complex blocks, A1 m1 x n and A2 m2 x n,
 * m1, m2 >= n (the paper's general setting, Sec. 1): U1 (m1 x n) and U2
 * (m2 x n) with orthonormal columns, V1 (n x n).  The real embeddings
 * (2 m_i x 2n) are reduced by Householder QRs E_i = Q_i R_i, the square real
 * path runs on [R1; R2] and U_i = Q_i U_i', then the complex factors are read
 * back as for zcsd_zcsd.  Interleaved complex column-major arrays as there:
 * d_A1 (ld >= m1), d_A2 (ld >= m2) read only; d_U1 (ld >= m1), d_U2
 * (ld >= m2), d_V1 (ld >= n), d_theta (n reals) written, the first
 * info->rank columns / entries valid.  Errors: ZCSD_EINVAL for n < 1,
 * m_i < n, m_i > 32767, NULL pointers, short leading dimensions or another
 * precision; otherwise as zcsd_zcsd.
 */
zcsd_status zcsd_zcsd_mn(zcsd_handle* handle, int m1, int m2, int n,
                         const double* d_A1, int lda1, const double* d_A2, int lda2,
                         double* d_U1, int ldu1, double* d_U2, int ldu2,
                         double* d_V1, int ldv1, double* d_theta,
                         const zcsd_opts* opts, zcsd_info* info);

/*
 * Complete 2 x 2 CS decomposition of an orthogonal 2n x 2n matrix
 * A = [A1 A3; A2 A4] (Remark (viii) of Sec. 3):
 *    A = diag(U1, U2) [C -S; S C] diag(V1, V2)^T,  C = diag(cos theta),
 *    S = diag(sin theta), 0 <= theta_1 <= ... <= theta_n <= pi/2.
 * Algorithm 1 on the first block column [A1; A2] gives U1, U2, V1 and theta;
 * then X = -A3^T U1 S + A4^T U2 C and V2 is the Q factor of X = QR with
 * diag(R) >= 0 (X itself is orthogonal when A is).  All blocks n x n,
 * column-major device memory owned by the caller (ld >= n); d_theta has
 * length n.  opts may be NULL (defaults; rank_mode ZCSD_RANK_DEFICIENT is
 * rejected with ZCSD_EINVAL); info may be NULL.  Returns ZCSD_ENOTISO when
 * [A1; A2] is detected rank deficient (A is then not orthogonal).
 */
zcsd_status zcsd_dcsd2x2(zcsd_handle* handle, int n,
                         const double* d_A1, int lda1, const double* d_A2, int lda2,
                         const double* d_A3, int lda3, const double* d_A4, int lda4,
                         double* d_U1, int ldu1, double* d_U2, int ldu2,
                         double* d_V1, int ldv1, double* d_V2, int ldv2, double* d_theta,
                         const zcsd_opts* opts, zcsd_info* info);

/*
 * Batched CS decomposition of `batch` independent problems of different sizes
 * (Algorithm 1, or Algorithm 3 for problems detected or forced rank-deficient;
 * the same outputs and conventions as zcsd_dcsd per problem).  Packed ragged
 * layout: problem k has size n_host[k] (1..4096) and its n_k x n_k blocks of
 * A1, A2 (inputs) and U1, U2, V1 (outputs) start at element offset
 * off_host[k] of the respective device array, column-major with ld = n_k;
 * its angles start at element sum_{j<k} n_j of d_theta.  Only the first
 * rank_host[k] columns / angles of a problem are valid, the rest are zero.
 * n_host, off_host (read) and rank_host (written) are host arrays of length
 * batch; matrices are device memory owned by the caller and outputs must not
 * alias inputs.  Problems are grouped into padded size classes that run
 * through the batched kernels together; padding is decoupled from the real
 * spectrum (identity in the polar factors, an isolated eigenvalue 3 in B), so
 * results equal zcsd_dcsd's up to rounding.  Synchronous on the handle's
 * stream.  Errors: ZCSD_EINVAL (bad sizes/offsets/pointers, batch outside
 * 1..65535, opts out of range: mu must lie in (1, 3)); ZCSD_ENOTISO /
 * ZCSD_ENOCONV / ZCSD_ENOMEM as zcsd_dcsd.  info (may be NULL) holds the
 * largest r used, the deepest Zolo-eig level count, the total splits and, in
 * info->repair, the number of problems whose polar factor Algorithm 2 replaced.
 * A size class of full-rank problems shares one lower bound l of sigma_min;
 * when it reaches eps (a member may have sigma_min(A_i) < eps, Sec. 5.1), the
 * class's problems run one at a time through the single path of zcsd_dcsd,
 * which has the repair of Algorithm 2, instead of the batched kernels.
 * Small full-rank problems (n <= ZCSD_TUNE_ONE_WORKGROUP_MAX_N) run instead
 * as one workgroup each, with their own l and their Zolotarev coefficients
 * from a table of lower bounds (0.9 * 10^(-q/8), the largest one <= l); one
 * whose l reaches eps also goes to the single path.
 */
zcsd_status zcsd_dcsd_batched(zcsd_handle* handle, int batch, const int* n_host,
                              const long long* off_host,
                              const double* d_A1, const double* d_A2,
                              double* d_U1, double* d_U2, double* d_V1, double* d_theta,
                              int* rank_host, const zcsd_opts* opts, zcsd_info* info);

/*
 * Batched CS decompositions of small full-rank problems with every decision
 * on the device, for HIP graph capture (Algorithm 1 with Zolo-pd, Sec. 5,
 * and the Jacobi solve of Zolo-eig's blocks, Sec. 5): each problem runs as
 * one workgroup with its own lower bound l and the Zolotarev coefficients of
 * the largest tabulated bound 0.9 * 10^(-q/8) <= l, as the one-workgroup
 * problems of zcsd_dcsd_batched do.  The call enqueues, on the handle's
 * stream, one kernel that sorts the problems by descending size (a counting
 * sort in one workgroup), so that each tier of sizes (49..64, 33..48, 17..32,
 * 1..16) is a contiguous range of the list, and four persistent launches that
 * read their ranges from the device; it makes no host transfer,
 * synchronisation, memset or allocation, so a captured graph replays it over
 * new contents of the same buffers.
 * All arrays are device memory owned by the caller, read at run time:
 *  d_n[k]      size n_k of problem k (1..64; any other size gets status 3);
 *  d_off[k]    element offset of problem k's n_k x n_k blocks in d_A1, d_A2
 *              (inputs) and d_U1, d_U2, d_V1 (outputs), column-major, ld n_k;
 *  d_toff[k]   element offset of its n_k angles in d_theta (ascending);
 *  d_status[k] written: low byte 0 = outputs written, 1 = the l estimate
 *              reached opts->eps (sigma_min(A_i) below it or a rank-deficient
 *              member: outputs not written; zcsd_dcsd_batched handles such
 *              members, with Algorithm 2 or 3), 2 = a Cholesky factorisation
 *              broke down (not written), 3 = size outside 1..64 (not
 *              written); bits 8.. the Zolotarev degree used;
 *  d_ws        workspace of at least the size zcsd_small_batch_prepare
 *              returns for this batch, 256-byte aligned; its contents need
 *              no initialisation and are not meaningful afterwards.
 * Outputs must not alias inputs; problems' output blocks must not overlap.
 * The offsets live on the device and are not checked: every problem's blocks
 * and angles must lie inside the caller's arrays.
 * opts (may be NULL): eps, tol and postprocess as zcsd_dcsd; prec must be
 * ZCSD_FP64, r_override and ell_override 0, rank_mode not
 * ZCSD_RANK_DEFICIENT.  Errors (nothing enqueued): ZCSD_EINVAL for batch
 * outside 1..2^20, NULL pointers, a short or misaligned workspace, options
 * outside the above, or no prior zcsd_small_batch_prepare for these eps and
 * tol on the handle's device.  Calls that share a workspace must not overlap
 * in time.
 */
zcsd_status zcsd_dcsd_batched_small(zcsd_handle* handle, int batch, const int* d_n,
                                    const long long* d_off, const long long* d_toff,
                                    const double* d_A1, const double* d_A2,
                                    double* d_U1, double* d_U2, double* d_V1, double* d_theta,
                                    int* d_status, void* d_ws, size_t ws_bytes,
                                    const zcsd_opts* opts);
/*
 * Set-up of zcsd_dcsd_batched_small, outside any capture: uploads the
 * Zolotarev coefficient table of (opts->eps, opts->tol) to the handle's device
 * once (synchronous; kept until the process ends, a few KB) and returns in
 * *ws_bytes the workspace a call with `batch` problems needs (4 batch bytes
 * of list plus the scratch of the persistent grids, about 57 MB on 256
 * compute units).  Errors: ZCSD_EINVAL as zcsd_dcsd_batched_small (or a
 * NULL ws_bytes); ZCSD_EHIP if the table cannot be allocated or copied.
 */
zcsd_status zcsd_small_batch_prepare(zcsd_handle* handle, int batch, const zcsd_opts* opts,
                                     size_t* ws_bytes);

/*
 * Backward of `batch` full-rank CS decompositions of size n: the gradients
 * gA1, gA2 of L = sum_i g_theta[i] theta_i + <G_W1, W1> + <G_W2, W2> with
 * respect to A1 and A2, where W_i = U_i V1^T are the polar factors of
 * Algorithm 1 and theta its angles (with Remark (iii)).
 * First-order perturbation of c_i = v_i^T H1 v_i and s_i = v_i^T H2 v_i gives
 * d theta_i = -s_i u1_i^T dA1 v_i + c_i u2_i^T dA2 v_i; the polar factor of
 * A = U Sigma V^T moves by U [(E - E^T)/(sigma_j + sigma_k)] V^T, E = U^T dA V.
 * Inputs are the outputs of zcsd_dcsd: d_U1, d_U2, d_V1 (n x n, ld n, batch
 * stride n*n) and d_theta (batch stride n), column-major, device memory,
 * caller-owned and read only.  d_g_theta (stride n), d_G_W1, d_G_W2 (n x n,
 * stride n*n) may each be NULL (zero).  d_gA1, d_gA2 (n x n, stride n*n) are
 * written; they must not alias the inputs.  Pairs of zero singular values
 * (rank-deficient inputs) contribute zero.  Synchronous on the handle's stream.
 * Errors: ZCSD_EINVAL for non-positive sizes, batch > 65535 or a NULL
 * required pointer (nothing enqueued); ZCSD_ENOMEM if the workspace
 * (2 batch n^2 doubles) cannot be allocated.
 */
zcsd_status zcsd_dcsd_backward(zcsd_handle* handle, int batch, int n,
                               const double* d_U1, const double* d_U2, const double* d_V1,
                               const double* d_theta, const double* d_g_theta,
                               const double* d_G_W1, const double* d_G_W2,
                               double* d_gA1, double* d_gA2);

/*
 * zcsd_dcsd_backward that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, layout, ownership and results as
 * zcsd_dcsd_backward.  Its intermediates (2 n^2 doubles per problem) live in
 * a fixed device array of 2^23 doubles (64 MiB) that the library holds on
 * every device it runs on until the process ends; the batch is processed in
 * passes of floor(2^23 / (2 n^2)) problems.  Limit: n <= 2048 (ZCSD_EINVAL
 * beyond it, nothing enqueued).  Asynchronous: returns once the work is
 * enqueued on the handle's stream, with no allocation, synchronisation or
 * host transfer.  Every call on a device shares that device's array: calls
 * that overlap in time on one device (on different streams or handles) race
 * with each other; calls on one stream are ordered.  Nothing left in the
 * array by an earlier call is read (every element is written before use).
 */
zcsd_status zcsd_dcsd_backward_noalloc(zcsd_handle* handle, int batch, int n,
                                       const double* d_U1, const double* d_U2, const double* d_V1,
                                       const double* d_theta, const double* d_g_theta,
                                       const double* d_G_W1, const double* d_G_W2,
                                       double* d_gA1, double* d_gA2);

/*
 * Batched Zolo-pd (Sec. 5): polar decompositions X_b = W_b H_b of `batch`
 * n x n matrices stored at d_X + b*strideX (ld ldx), scaled by 1/alpha (alpha
 * must bound sigma_max).  One shared lower bound l (estimated as the minimum
 * over the batch of 1/‖R_b^{-1}‖_F, or opts->ell_override) and degree r
 * (opts->r_override or the smallest r <= 8 with 1 - l_2 <= opts->tol).
 * Outputs W (ld n, stride n*n), H = sym(W^T X) (ld n, stride n*n; may be
 * NULL), and optionally the first iterate X1 (may be NULL).
 */
zcsd_status zcsd_dzolo_pd(zcsd_handle* handle, int batch, int n, double alpha,
                          const double* d_X, int ldx, long long strideX,
                          double* d_W, double* d_H, double* d_X1,
                          const zcsd_opts* opts, zcsd_info* info);

/*
 * Symmetric eigendecomposition B = V diag(lambda) V^T of an n x n symmetric
 * matrix by Zolo-eig (Sec. 5: spectral divide and conquer on the sign
 * function computed by Zolo-pd, Jacobi on blocks of at most opts->n_leaf).
 * lo <= lambda_min and hi >= lambda_max must bound the spectrum.  lambda is
 * returned in ascending order with the matching columns of V (ld ldv).
 */
zcsd_status zcsd_dsyev_zolo(zcsd_handle* handle, int n, const double* d_B, int ldb,
                            double lo, double hi, double* d_V, int ldv, double* d_lambda,
                            const zcsd_opts* opts, zcsd_info* info);

/*
 * Zolotarev coefficients of one iteration (host only): c[0..2r-1] = c_1..c_2r,
 * a[0..r-1], M with Z(1) = 1, and l_next = Z(l) (Sec. 5; definitions in the
 * library's host code).  Returns ZCSD_EINVAL unless 0 < l <= 1 and 1 <= r <= 8.
 */
zcsd_status zcsd_zolo_coeffs(double ell, int r, double* h_c, double* h_a, double* h_M,
                             double* h_ell_next);
/* Smallest r in 1..8 with 1 - l_2 <= tol after two iterations from l, or 0 if none. */
int zcsd_zolo_choose_r(double ell, double tol);

/*
 * FP64 MFMA matrix product (the building block of every step above):
 * C_b = alpha op(A_b) op(B_b) + beta C_b for b < batch, op = transpose when
 * transA/transB != 0; op(A) is m x k, op(B) is k x n; batch strides in elements.
 */
zcsd_status zcsd_dgemm(zcsd_handle* handle, int transA, int transB, int m, int n, int k,
                       double alpha, const double* d_A, int lda, long long strideA,
                       const double* d_B, int ldb, long long strideB, double beta,
                       double* d_C, int ldc, long long strideC, int batch);
/* The same product with A and B rounded to FP32 and FP32 accumulation on the
 * FP32 matrix cores (v_mfma_f32_16x16x4f32), FP64 in and out: the products of
 * the mixed-precision mode's Zolo-eig.  Same arguments and errors as zcsd_dgemm. */
zcsd_status zcsd_dgemm_f32acc(zcsd_handle* handle, int transA, int transB, int m, int n, int k,
                              double alpha, const double* d_A, int lda, long long strideA,
                              const double* d_B, int ldb, long long strideB, double beta,
                              double* d_C, int ldc, long long strideC, int batch);

/*
 * The product with the structure options the path uses internally (exported
 * for testing; same arguments and errors as zcsd_dgemm, plus):
 *  flags: ZCSD_GEMM_SYM_UPPER   symmetric product (m == n, beta == 0): only
 *                               the tiles of C on or above the diagonal are
 *                               computed, the others keep their contents
 *                               (every entry i <= j is computed);
 *         ZCSD_GEMM_UPPER_ONLY  only the upper triangle of C is wanted (m == n,
 *                               any beta): tiles below the diagonal are skipped;
 *         ZCSD_GEMM_F32ACC      FP32 matrix cores (as zcsd_dgemm_f32acc);
 *  tri, kseg: triangular operands; K is made of k / kseg segments (kseg must
 *         divide k), and within each segment, counting k from its start,
 *         op(A) is upper (tri & 1: zero for k < i) or lower (tri & 2: zero for
 *         k > i) and op(B) upper (tri & 4: zero for k > j) or lower (tri & 8:
 *         zero for k < j); products the structure makes zero are skipped, so
 *         those zeros must be present in memory (0: dense);
 *  d_ws, ws_elems: optional device workspace (caller-owned) for the
 *         deterministic split of k across workgroups in products with few
 *         output tiles and k >= 1024; NULL / 0 for none.
 * ZCSD_EINVAL for unknown flags, tri outside 0..15, a kseg that does not
 * divide k, or ZCSD_GEMM_SYM_UPPER with m != n or beta != 0.
 */
enum { ZCSD_GEMM_SYM_UPPER = 1, ZCSD_GEMM_UPPER_ONLY = 2, ZCSD_GEMM_F32ACC = 4 };
zcsd_status zcsd_dgemm_ex(zcsd_handle* handle, int transA, int transB, int m, int n, int k,
                          double alpha, const double* d_A, int lda, long long strideA,
                          const double* d_B, int ldb, long long strideB, double beta,
                          double* d_C, int ldc, long long strideC, int batch, int flags,
                          int tri, int kseg, double* d_ws, size_t ws_elems);

/*
 * Blocked Householder QR (the QR form of Zolo-pd, Sec. 5), batched in place.
 * stacked == 0: d_M_b is m x n (m >= n); on return its top n x n upper triangle
 *   holds R and everything below is zero; d_Q_b (m x n, may be NULL) receives
 *   the explicit Q with Q R = M.
 * stacked != 0: d_M_b is the 2n x n matrix [R0; D] with R0 upper triangular and
 *   D diagonal (m must equal 2n); the structured factorisation touches only the
 *   nonzero pattern; outputs as above.
 */
zcsd_status zcsd_dqr(zcsd_handle* handle, int batch, int stacked, int m, int n,
                     double* d_M, int ldm, long long strideM,
                     double* d_Q, int ldq, long long strideQ);

/*
 * Kernel timing for measurement tools.  Between zcsd_profile_begin() and
 * zcsd_profile_end(), every launch of the instrumented kernels (the MFMA GEMM
 * tile variants, the QR panel, the Cholesky base, the Jacobi leaf) is
 * bracketed by HIP events on its own stream and its algorithmic flops and
 * bytes are added to a record named after the kernel (for example
 * "dgemm_128x128_NT").  zcsd_profile_query fills the launch count, the
 * summed algorithmic flops and bytes and the summed event time in ms of one
 * record and returns 1, or returns 0 if there is none; it synchronises on the
 * recorded events.  zcsd_profile_names writes the record names, one per line,
 * into buf (NUL-terminated, truncated to len) and returns the full length.
 * zcsd_profile_filter restricts recording to one record so that the event
 * pairs perturb nothing else.  Process-wide, not thread-safe with respect to
 * concurrent begin/end.
 */
void zcsd_profile_begin(void);
void zcsd_profile_end(void);
/* Restrict recording to the record `name` (NULL: record every kernel). */
void zcsd_profile_filter(const char* name);
int zcsd_profile_query(const char* name, long long* launches, double* flops, double* bytes,
                       double* ms);
int zcsd_profile_names(char* buf, int len);

#ifdef __cplusplus
}
#endif
#endif /* ZCSD_H */
