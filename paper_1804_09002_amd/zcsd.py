"""ctypes binding of libzcsd (argument marshalling only).

Every step of the decomposition runs in the HIP library; this module only
checks shapes, passes device pointers of torch tensors, and converts between
the user's (rows, cols) indexing and the library's column-major storage:
a matrix X is handed to the library as the contiguous buffer of ``X.t()``,
and results come back as ``.t()`` views of column-major buffers.

If ``libzcsd.so`` is missing or no HIP device is visible, every call raises;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libzcsd.so")

ZCSD_OK, ZCSD_EINVAL, ZCSD_ENOTISO, ZCSD_ENOCONV, ZCSD_EREPAIR, ZCSD_EHIP, ZCSD_ENOMEM = range(7)
RANK_AUTO, RANK_FULL, RANK_DEFICIENT = 0, 1, 2
FP64, MIXED_FP32 = 0, 1


class ZcsdError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {_lib().zcsd_status_string(status).decode()}")


class Opts(C.Structure):
    _fields_ = [("prec", C.c_int), ("rank_mode", C.c_int), ("eps", C.c_double),
                ("mu", C.c_double), ("tol", C.c_double), ("r_override", C.c_int),
                ("ell_override", C.c_double), ("n_leaf", C.c_int), ("postprocess", C.c_int)]


class Info(C.Structure):
    _fields_ = [("rank", C.c_int), ("r_used", C.c_int * 2), ("ell", C.c_double * 2),
                ("zolo_resid", C.c_double), ("eig_levels", C.c_int), ("eig_splits", C.c_int),
                ("eig_max_r", C.c_int), ("eig_offblock", C.c_double),
                ("eig_coupling", C.c_double), ("eig_full_refinements", C.c_int),
                ("lowp_products", C.c_int), ("repair", C.c_int), ("repair_resid", C.c_double),
                ("time_ms", C.c_double * 4)]

    def as_dict(self):
        return {"rank": self.rank, "r_used": list(self.r_used), "ell": list(self.ell),
                "zolo_resid": self.zolo_resid, "eig_levels": self.eig_levels,
                "eig_splits": self.eig_splits, "eig_max_r": self.eig_max_r,
                "eig_offblock": self.eig_offblock, "eig_coupling": self.eig_coupling,
                "eig_full_refinements": self.eig_full_refinements,
                "lowp_products": self.lowp_products, "repair": self.repair,
                "repair_resid": self.repair_resid,
                "time_ms": list(self.time_ms)}


_L = None


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"libzcsd.so not built ({_LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(_LIB_PATH)
        vp, i, d, ll = C.c_void_p, C.c_int, C.c_double, C.c_longlong
        L.zcsd_create.argtypes = [C.POINTER(vp), i]
        L.zcsd_destroy.argtypes = [vp]
        L.zcsd_set_stream.argtypes = [vp, vp]
        L.zcsd_default_opts.argtypes = [C.POINTER(Opts)]
        L.zcsd_default_opts.restype = None
        L.zcsd_status_string.argtypes = [i]
        L.zcsd_status_string.restype = C.c_char_p
        L.zcsd_dgemm.argtypes = [vp, i, i, i, i, i, d, vp, i, ll, vp, i, ll, d, vp, i, ll, i]
        if hasattr(L, "zcsd_dgemm_f32acc"):
            L.zcsd_dgemm_f32acc.argtypes = L.zcsd_dgemm.argtypes
        if hasattr(L, "zcsd_dgemm_ex"):
            L.zcsd_dgemm_ex.argtypes = L.zcsd_dgemm.argtypes + [i, i, i, vp, C.c_size_t]
        for name, args in {
            "zcsd_dcsd": [vp, i, vp, i, vp, i, vp, i, vp, i, vp, i, vp, vp, vp,
                          C.POINTER(Opts), C.POINTER(Info)],
            "zcsd_dcsd2x2": [vp, i, vp, i, vp, i, vp, i, vp, i, vp, i, vp, i, vp, i, vp, i, vp,
                             C.POINTER(Opts), C.POINTER(Info)],
            "zcsd_dcsd_mn": [vp, i, i, i, vp, i, vp, i, vp, i, vp, i, vp, i, vp,
                             C.POINTER(Opts), C.POINTER(Info)],
            "zcsd_zcsd": [vp, i, vp, i, vp, i, vp, i, vp, i, vp, i, vp,
                          C.POINTER(Opts), C.POINTER(Info)],
            "zcsd_zcsd_mn": [vp, i, i, i, vp, i, vp, i, vp, i, vp, i, vp, i, vp,
                             C.POINTER(Opts), C.POINTER(Info)],
            "zcsd_dzolo_pd": [vp, i, i, d, vp, i, ll, vp, vp, vp, C.POINTER(Opts), C.POINTER(Info)],
            "zcsd_dsyev_zolo": [vp, i, vp, i, d, d, vp, i, vp, C.POINTER(Opts), C.POINTER(Info)],
            "zcsd_dcsd_backward": [vp, i, i, vp, vp, vp, vp, vp, vp, vp, vp, vp],
            "zcsd_dcsd_backward_noalloc": [vp, i, i, vp, vp, vp, vp, vp, vp, vp, vp, vp],
            "zcsd_dcsd_batched": [vp, i, C.POINTER(C.c_int), C.POINTER(C.c_longlong), vp, vp, vp, vp,
                                  vp, vp, C.POINTER(C.c_int), C.POINTER(Opts), C.POINTER(Info)],
            "zcsd_zolo_coeffs": [d, i, C.POINTER(d), C.POINTER(d), C.POINTER(d), C.POINTER(d)],
            "zcsd_small_batch_prepare": [vp, i, C.POINTER(Opts), C.POINTER(C.c_size_t)],
            "zcsd_dcsd_batched_small": [vp, i, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t,
                                        C.POINTER(Opts)],
            "zcsd_set_tuning": [vp, i, i],
            "zcsd_get_tuning": [vp, i, C.POINTER(C.c_int)],
            "zcsd_zolo_choose_r": [d, d],
            "zcsd_workspace_size": [vp, i, C.POINTER(Opts), C.POINTER(C.c_size_t)],
            "zcsd_dqr": [vp, i, i, i, i, vp, i, ll, vp, i, ll],
            "zcsd_profile_query": [C.c_char_p, C.POINTER(ll), C.POINTER(d), C.POINTER(d), C.POINTER(d)],
            "zcsd_profile_names": [C.c_char_p, i],
            "zcsd_profile_filter": [C.c_char_p],
        }.items():
            if hasattr(L, name):
                getattr(L, name).argtypes = args
        if hasattr(L, "zcsd_zolo_choose_r"):
            L.zcsd_zolo_choose_r.restype = C.c_int
        # the struct layouts above must be the library's: a smaller Info would
        # let the library write past it
        L.zcsd_sizeof_opts.restype = C.c_size_t
        L.zcsd_sizeof_info.restype = C.c_size_t
        if (L.zcsd_sizeof_opts() != C.sizeof(Opts) or L.zcsd_sizeof_info() != C.sizeof(Info)):
            raise RuntimeError(f"{_LIB_PATH} was built with other zcsd_opts/zcsd_info layouts "
                               f"({L.zcsd_sizeof_opts()}/{L.zcsd_sizeof_info()} bytes, binding "
                               f"{C.sizeof(Opts)}/{C.sizeof(Info)}); rebuild it")
        _L = L
    return _L


def lib():
    return _lib()


def workspace_size(n, **opts):
    """Device bytes a square CSD of size n reserves (zcsd_workspace_size; host only)."""
    o = default_opts(**opts)
    b = C.c_size_t(0)
    _check(_lib().zcsd_workspace_size(None, int(n), C.byref(o), C.byref(b)), "zcsd_workspace_size")
    return int(b.value)


def _check(st, what):
    if st != ZCSD_OK:
        raise ZcsdError(st, what)


_HANDLES = {}


def handle(device=None):
    """Per-device library handle bound to torch's current stream at call time."""
    if not torch.cuda.is_available():
        raise RuntimeError("zcsd: no HIP device visible")
    dev = torch.cuda.current_device() if device is None else int(device)
    h = _HANDLES.get(dev)
    if h is None:
        h = C.c_void_p()
        _check(_lib().zcsd_create(C.byref(h), dev), "zcsd_create")
        _HANDLES[dev] = h
    _lib().zcsd_set_stream(h, C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    return h


(TUNE_BATCHED_WORKERS, TUNE_CLASS_STEP_SMALL, TUNE_CLASS_STEP_MID, TUNE_CLASS_STEP_LARGE,
 TUNE_ONE_WORKGROUP_MAX_N, TUNE_GEMM_TILE128_MIN) = range(6)
TUNE_KEYS = {"batched_workers": TUNE_BATCHED_WORKERS, "class_step_small": TUNE_CLASS_STEP_SMALL,
             "class_step_mid": TUNE_CLASS_STEP_MID, "class_step_large": TUNE_CLASS_STEP_LARGE,
             "one_workgroup_max_n": TUNE_ONE_WORKGROUP_MAX_N,
             "gemm_tile128_min": TUNE_GEMM_TILE128_MIN}


def set_tuning(device=None, **values):
    """Batched-path tuning of the device's handle (zcsd_set_tuning), e.g.
    set_tuning(batched_workers=4, class_step_small=8, class_step_mid=16,
    one_workgroup_max_n=64)."""
    h = handle(device)
    for k, v in values.items():
        _check(_lib().zcsd_set_tuning(h, TUNE_KEYS[k], int(v)), f"zcsd_set_tuning({k}={v})")


def get_tuning(device=None):
    """The batched-path tuning of the device's handle, as a dict."""
    h = handle(device)
    out = {}
    for k, key in TUNE_KEYS.items():
        v = C.c_int(0)
        _check(_lib().zcsd_get_tuning(h, key, C.byref(v)), "zcsd_get_tuning")
        out[k] = v.value
    return out


def default_opts(**kw):
    o = Opts()
    _lib().zcsd_default_opts(C.byref(o))
    for k, v in kw.items():
        if v is None:
            continue
        if k == "rank_mode" and isinstance(v, str):
            v = {"auto": RANK_AUTO, "full": RANK_FULL, "deficient": RANK_DEFICIENT}[v]
        if k == "prec" and isinstance(v, str):
            v = {"fp64": FP64, "mixed_fp32": MIXED_FP32}[v]
        setattr(o, k, v)
    return o


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _colmajor(X, name):
    """(rows, cols) float64 CUDA tensor -> contiguous column-major buffer (cols, rows)."""
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float64 and X.dim() == 2):
        raise TypeError(f"{name} must be a 2-D float64 tensor on a HIP device")
    return X.t().contiguous()


def dgemm(A, B, transA=False, transB=False, alpha=1.0, beta=0.0, C_=None, f32acc=False):
    """C = alpha op(A) op(B) + beta C for 2-D or batched 3-D float64 device tensors (row-major API).

    f32acc=True runs the product on the FP32 matrix cores (zcsd_dgemm_f32acc)."""
    batched = A.dim() == 3
    if not batched:
        A, B = A.unsqueeze(0), B.unsqueeze(0)
        C_ = None if C_ is None else C_.unsqueeze(0)
    # column-major views: a row-major (r, c) tensor is the column-major (c, r) matrix = X^T.
    # C = op(A) op(B)  <=>  C^T = op(B)^T op(A)^T: call the library with the roles swapped.
    Ab, Bb = A.contiguous(), B.contiguous()
    bs, ar, ac = Ab.shape
    _, br, bc = Bb.shape
    m_ = ac if transA else ar
    k_ = ar if transA else ac
    n_ = br if transB else bc
    out = torch.empty((bs, m_, n_), dtype=torch.float64, device=A.device) if C_ is None else C_.contiguous()
    h = handle(A.device.index)
    # library computes (col-major) C' = op'(B') op'(A') with X' = X^T storage
    fn = _lib().zcsd_dgemm_f32acc if f32acc else _lib().zcsd_dgemm
    st = fn(h, 1 if transB else 0, 1 if transA else 0, n_, m_, k_, alpha,
            _ptr(Bb), bc, br * bc, _ptr(Ab), ac, ar * ac, beta,
            _ptr(out), n_, m_ * n_, bs)
    _check(st, "zcsd_dgemm")
    return out if batched else out[0]


GEMM_SYM_UPPER, GEMM_UPPER_ONLY, GEMM_F32ACC = 1, 2, 4


def dgemm_ex(A, B, C_, transA, transB, m, n, k, alpha=1.0, beta=0.0, flags=0, tri=0, kseg=0,
             ws=None):
    """zcsd_dgemm_ex on column-major buffers (the library's own layout).

    A, B, C_ are contiguous float64 device tensors of shape (batch, cols, rows):
    each [b] is the transpose of a column-major rows x cols matrix with
    leading dimension rows.  op(A) is m x k, op(B) k x n, C_ m x n.  ws is an
    optional flat float64 device tensor (split-K workspace)."""
    for X, nm in ((A, "A"), (B, "B"), (C_, "C")):
        if not (X.is_cuda and X.dtype == torch.float64 and X.dim() == 3 and X.is_contiguous()):
            raise TypeError(f"dgemm_ex: {nm} must be a contiguous (batch, cols, rows) float64 tensor")
    bs = C_.shape[0]
    h = handle(C_.device.index)
    st = _lib().zcsd_dgemm_ex(h, 1 if transA else 0, 1 if transB else 0, m, n, k, float(alpha),
                              _ptr(A), A.shape[2], A.shape[1] * A.shape[2],
                              _ptr(B), B.shape[2], B.shape[1] * B.shape[2], float(beta),
                              _ptr(C_), C_.shape[2], C_.shape[1] * C_.shape[2], bs,
                              int(flags), int(tri), int(kseg),
                              _ptr(ws) if ws is not None else None,
                              0 if ws is None else ws.numel())
    _check(st, "zcsd_dgemm_ex")
    return C_


def zolo_coeffs(ell, r):
    """Host Zolotarev coefficients from the library: (c[2r], a[r], M, ell_next)."""
    c = (C.c_double * (2 * r))()
    a = (C.c_double * r)()
    M = C.c_double()
    nx = C.c_double()
    _check(_lib().zcsd_zolo_coeffs(float(ell), int(r), c, a, C.byref(M), C.byref(nx)), "zcsd_zolo_coeffs")
    return list(c), list(a), M.value, nx.value


def zolo_choose_r(ell, tol=2.0 ** -53):
    return int(_lib().zcsd_zolo_choose_r(float(ell), float(tol)))


def zolo_pd(X, alpha=1.0, r=None, ell=None, want_H=True, want_X1=False):
    """Batched Zolo-pd of a (n, n) or (batch, n, n) float64 device tensor.

    Returns (W, H, X1, info) with the same leading shape (H / X1 None unless requested).
    """
    batched = X.dim() == 3
    Xb = X if batched else X.unsqueeze(0)
    bs, n, n2 = Xb.shape
    if n != n2:
        raise ValueError("zolo_pd: square matrices only")
    Xc = Xb.transpose(1, 2).contiguous()          # column-major buffers
    W = torch.empty_like(Xc)
    H = torch.empty_like(Xc) if want_H else None
    X1 = torch.empty_like(Xc) if want_X1 else None
    o = default_opts(r_override=r or 0, ell_override=ell or 0.0)
    info = Info()
    h = handle(X.device.index)
    st = _lib().zcsd_dzolo_pd(h, bs, n, float(alpha), _ptr(Xc), n, n * n, _ptr(W),
                              _ptr(H) if H is not None else None, _ptr(X1) if X1 is not None else None,
                              C.byref(o), C.byref(info))
    _check(st, "zcsd_dzolo_pd")
    tr = lambda T: None if T is None else (T.transpose(1, 2) if batched else T[0].t())
    return tr(W), tr(H), tr(X1), info.as_dict()


def qr(M, stacked=False, want_q=True):
    """Batched blocked Householder QR of (m, n) / (batch, m, n) device tensors.

    Returns (R, Q): R (n, n) upper triangular, Q (m, n); stacked=True expects [R0; D] (2n x n).
    """
    batched = M.dim() == 3
    Mb = M if batched else M.unsqueeze(0)
    bs, m, n = Mb.shape
    Mc = Mb.transpose(1, 2).contiguous()
    Q = torch.empty_like(Mc) if want_q else None
    h = handle(M.device.index)
    st = _lib().zcsd_dqr(h, bs, 1 if stacked else 0, m, n, _ptr(Mc), m, m * n,
                         _ptr(Q) if Q is not None else None, m, m * n)
    _check(st, "zcsd_dqr")
    R = Mc.transpose(1, 2)[:, :n, :]
    Qr = None if Q is None else Q.transpose(1, 2)
    if not batched:
        R = R[0]
        Qr = None if Qr is None else Qr[0]
    return R, Qr


def syev_zolo(B, lo=-1.0, hi=1.0, n_leaf=None):
    """Zolo-eig of a symmetric (n, n) float64 device tensor: (lambda ascending, V, info)."""
    n = B.shape[0]
    Bc = _colmajor(B, "B")
    V = torch.empty_like(Bc)
    lam = torch.empty(n, dtype=torch.float64, device=B.device)
    o = default_opts(n_leaf=n_leaf)
    info = Info()
    h = handle(B.device.index)
    st = _lib().zcsd_dsyev_zolo(h, n, _ptr(Bc), n, float(lo), float(hi), _ptr(V), n, _ptr(lam),
                                C.byref(o), C.byref(info))
    _check(st, "zcsd_dsyev_zolo")
    return lam, V.t(), info.as_dict()


def csd(A1, A2, rank_mode="auto", r=None, ell=None, want_polar=False, **opts):
    """CS decomposition of [A1; A2] (A1: (m1, n), A2: (m2, n) float64 HIP tensors, m1, m2 >= n).

    Returns (U1, U2, V1, theta, info) with A1 = U1 diag(cos theta) V1^T and
    A2 = U2 diag(sin theta) V1^T; in the rank-deficient case only the first
    info['rank'] columns / entries are valid (the rest are zero).  With
    want_polar=True (square blocks only), info also holds the polar factors
    'W1', 'W2'.  Square blocks use zcsd_dcsd, rectangular ones zcsd_dcsd_mn.
    Other keyword options are zcsd_opts fields, e.g. prec="mixed_fp32",
    postprocess=2 (angles from sin(theta) - cos(theta) = Lambda, Remark (iv)).
    """
    if A1.dim() != 2 or A2.dim() != 2 or A1.shape[1] != A2.shape[1]:
        raise ValueError("csd: A1 and A2 must be 2-D with the same number of columns")
    m1, n = A1.shape
    m2 = A2.shape[0]
    if (m1, m2) != (n, n):
        if m1 < n or m2 < n:
            raise ValueError("csd: need m1, m2 >= n")
        if want_polar:
            raise ValueError("csd: want_polar needs square blocks")
        a1 = _colmajor(A1, "A1")
        a2 = _colmajor(A2, "A2")
        U1 = torch.empty((n, m1), dtype=torch.float64, device=A1.device)
        U2 = torch.empty((n, m2), dtype=torch.float64, device=A1.device)
        V1 = torch.empty((n, n), dtype=torch.float64, device=A1.device)
        th = torch.empty(n, dtype=torch.float64, device=A1.device)
        o = default_opts(rank_mode=rank_mode, r_override=r or 0, ell_override=ell or 0.0, **opts)
        info = Info()
        h = handle(A1.device.index)
        st = _lib().zcsd_dcsd_mn(h, m1, m2, n, _ptr(a1), m1, _ptr(a2), m2, _ptr(U1), m1, _ptr(U2),
                                 m2, _ptr(V1), n, _ptr(th), C.byref(o), C.byref(info))
        _check(st, "zcsd_dcsd_mn")
        return U1.t(), U2.t(), V1.t(), th, info.as_dict()
    a1 = _colmajor(A1, "A1")
    a2 = _colmajor(A2, "A2")
    U1 = torch.empty_like(a1)
    U2 = torch.empty_like(a1)
    V1 = torch.empty_like(a1)
    th = torch.empty(n, dtype=torch.float64, device=A1.device)
    W1 = torch.empty_like(a1) if want_polar else None
    W2 = torch.empty_like(a1) if want_polar else None
    o = default_opts(rank_mode=rank_mode, r_override=r or 0, ell_override=ell or 0.0, **opts)
    info = Info()
    h = handle(A1.device.index)
    st = _lib().zcsd_dcsd(h, n, _ptr(a1), n, _ptr(a2), n, _ptr(U1), n, _ptr(U2), n, _ptr(V1), n,
                          _ptr(th), _ptr(W1) if W1 is not None else None,
                          _ptr(W2) if W2 is not None else None, C.byref(o), C.byref(info))
    _check(st, "zcsd_dcsd")
    d = info.as_dict()
    if want_polar:
        d["W1"], d["W2"] = W1.t(), W2.t()
    return U1.t(), U2.t(), V1.t(), th, d


def csd_complex(A1, A2, rank_mode="auto", **opts):
    """CS decomposition of a complex [A1; A2] (A1: (m1, n), A2: (m2, n)
    complex128 HIP tensors, m1, m2 >= n).

    Returns (U1, U2, V1, theta, info) with A1 = U1 diag(cos theta) V1^H and
    A2 = U2 diag(sin theta) V1^H (complex128 factors, float64 theta); in the
    rank-deficient case only the first info['rank'] columns / entries are
    valid.  Computed through the real embedding of the blocks: zcsd_zcsd for
    square blocks, zcsd_zcsd_mn for rectangular ones.
    """
    for X, name in ((A1, "A1"), (A2, "A2")):
        if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.complex128
                and X.dim() == 2):
            raise TypeError(f"csd_complex: {name} must be a 2-D complex128 tensor on a HIP device")
    m1, n = A1.shape
    m2 = A2.shape[0]
    if A2.shape[1] != n or m1 < n or m2 < n:
        raise ValueError("csd_complex: need A1 (m1, n), A2 (m2, n) with m1, m2 >= n")
    a1 = A1.t().contiguous()
    a2 = A2.t().contiguous()
    dev = A1.device
    U1 = torch.empty((n, m1), dtype=torch.complex128, device=dev)
    U2 = torch.empty((n, m2), dtype=torch.complex128, device=dev)
    V1 = torch.empty((n, n), dtype=torch.complex128, device=dev)
    th = torch.empty(n, dtype=torch.float64, device=dev)
    o = default_opts(rank_mode=rank_mode, **opts)
    info = Info()
    h = handle(dev.index)
    if m1 == n and m2 == n:
        st = _lib().zcsd_zcsd(h, n, _ptr(a1), n, _ptr(a2), n, _ptr(U1), n, _ptr(U2), n, _ptr(V1), n,
                              _ptr(th), C.byref(o), C.byref(info))
        _check(st, "zcsd_zcsd")
    else:
        st = _lib().zcsd_zcsd_mn(h, m1, m2, n, _ptr(a1), m1, _ptr(a2), m2, _ptr(U1), m1, _ptr(U2), m2,
                                 _ptr(V1), n, _ptr(th), C.byref(o), C.byref(info))
        _check(st, "zcsd_zcsd_mn")
    return U1.t(), U2.t(), V1.t(), th, info.as_dict()


def csd2x2(A1, A2, A3, A4, **opts):
    """Complete 2 x 2 CSD of the orthogonal [A1 A3; A2 A4] (n x n float64 HIP tensors).

    Returns (U1, U2, V1, V2, theta, info) with
    A = diag(U1, U2) [C -S; S C] diag(V1, V2)^T (zcsd_dcsd2x2).
    """
    n = A1.shape[0]
    for X, name in ((A1, "A1"), (A2, "A2"), (A3, "A3"), (A4, "A4")):
        if X.shape != (n, n):
            raise ValueError(f"csd2x2: {name} must be n x n")
    a = [_colmajor(X, nm) for X, nm in ((A1, "A1"), (A2, "A2"), (A3, "A3"), (A4, "A4"))]
    U1, U2, V1, V2 = (torch.empty_like(a[0]) for _ in range(4))
    th = torch.empty(n, dtype=torch.float64, device=A1.device)
    o = default_opts(rank_mode=opts.pop("rank_mode", "auto"), **opts)
    info = Info()
    h = handle(A1.device.index)
    st = _lib().zcsd_dcsd2x2(h, n, _ptr(a[0]), n, _ptr(a[1]), n, _ptr(a[2]), n, _ptr(a[3]), n,
                             _ptr(U1), n, _ptr(U2), n, _ptr(V1), n, _ptr(V2), n, _ptr(th),
                             C.byref(o), C.byref(info))
    _check(st, "zcsd_dcsd2x2")
    return U1.t(), U2.t(), V1.t(), V2.t(), th, info.as_dict()


class profile:
    """Context manager: per-kernel HIP-event timing inside the library.

    with zcsd.profile(only="dgemm_128x128_NN") as p: ...; p.stats() -> {name: {...}}
    """

    def __init__(self, only=None):
        self.only = only

    def __enter__(self):
        L = _lib()
        L.zcsd_profile_filter(self.only.encode() if self.only else None)
        L.zcsd_profile_begin()
        return self

    def __exit__(self, *exc):
        _lib().zcsd_profile_end()
        return False

    @staticmethod
    def stats():
        L = _lib()
        n = L.zcsd_profile_names(None, 0)
        buf = C.create_string_buffer(n + 1)
        L.zcsd_profile_names(buf, n + 1)
        out = {}
        for name in buf.value.decode().split("\n"):
            if not name:
                continue
            la, fl, by, ms = C.c_longlong(), C.c_double(), C.c_double(), C.c_double()
            if L.zcsd_profile_query(name.encode(), C.byref(la), C.byref(fl), C.byref(by), C.byref(ms)):
                out[name] = {"launches": la.value, "flops": fl.value, "bytes": by.value, "ms": ms.value}
        return out


def _colmajor_batch(X, name, shape):
    """(batch, rows, cols) float64 device tensor -> contiguous column-major buffers."""
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float64 and X.dim() == 3
            and tuple(X.shape) == shape):
        raise TypeError(f"{name} must be a float64 HIP tensor of shape {shape}")
    return X.transpose(1, 2).contiguous()


def csd_backward(U1, U2, V1, theta, g_theta=None, G_W1=None, G_W2=None):
    """Gradients (gA1, gA2) of sum g_theta*theta + <G_W1, W1> + <G_W2, W2>.

    U1, U2, V1: (n, n) or (batch, n, n); theta, g_theta: (n,) or (batch, n); the
    decomposition must be full rank.  Any of g_theta, G_W1, G_W2 may be None.
    """
    return _csd_backward(U1, U2, V1, theta, g_theta, G_W1, G_W2, "zcsd_dcsd_backward")


def csd_backward_noalloc(U1, U2, V1, theta, g_theta=None, G_W1=None, G_W2=None):
    """csd_backward through zcsd_dcsd_backward_noalloc (no device allocation in
    the library, n <= 2048; enqueued on torch's current stream)."""
    return _csd_backward(U1, U2, V1, theta, g_theta, G_W1, G_W2, "zcsd_dcsd_backward_noalloc")


def _csd_backward(U1, U2, V1, theta, g_theta, G_W1, G_W2, entry):
    batched = U1.dim() == 3
    ex = (lambda t: t) if batched else (lambda t: None if t is None else t.unsqueeze(0))
    U1, U2, V1, theta, g_theta, G_W1, G_W2 = map(ex, (U1, U2, V1, theta, g_theta, G_W1, G_W2))
    bs, n, _ = U1.shape
    shp = (bs, n, n)
    u1, u2, v1 = (_colmajor_batch(X, nm, shp) for X, nm in ((U1, "U1"), (U2, "U2"), (V1, "V1")))
    g1 = None if G_W1 is None else _colmajor_batch(G_W1, "G_W1", shp)
    g2 = None if G_W2 is None else _colmajor_batch(G_W2, "G_W2", shp)
    if not (theta.is_cuda and theta.dtype == torch.float64 and tuple(theta.shape) == (bs, n)):
        raise TypeError("theta must be a float64 HIP tensor of shape (batch, n)")
    th = theta.contiguous()
    gt = None
    if g_theta is not None:
        if not (g_theta.is_cuda and g_theta.dtype == torch.float64 and tuple(g_theta.shape) == (bs, n)):
            raise TypeError("g_theta must be a float64 HIP tensor of shape (batch, n)")
        gt = g_theta.contiguous()
    gA1 = torch.empty_like(u1)
    gA2 = torch.empty_like(u1)
    h = handle(U1.device.index)
    st = getattr(_lib(), entry)(h, bs, n, _ptr(u1), _ptr(u2), _ptr(v1), _ptr(th),
                                _ptr(gt) if gt is not None else None,
                                _ptr(g1) if g1 is not None else None,
                                _ptr(g2) if g2 is not None else None, _ptr(gA1), _ptr(gA2))
    _check(st, entry)
    gA1, gA2 = gA1.transpose(1, 2), gA2.transpose(1, 2)
    return (gA1, gA2) if batched else (gA1[0], gA2[0])


class CSDFunction(torch.autograd.Function):
    """Differentiable CSD: (A1, A2) -> (U1, U2, V1, theta, W1, W2).

    theta and the polar factors W_i = U_i V1^T carry gradients (hand-written
    backward, zcsd_dcsd_backward); U1, U2, V1 are returned as non-differentiable
    (their columns are fixed only up to signs and rotations within equal angles).
    """

    @staticmethod
    def forward(ctx, A1, A2):
        U1, U2, V1, th, info = csd(A1, A2, want_polar=True)
        ctx.rank = info["rank"]
        ctx.save_for_backward(U1, U2, V1, th)
        W1, W2 = info["W1"], info["W2"]
        ctx.mark_non_differentiable(U1, U2, V1)
        return U1, U2, V1, th, W1, W2

    @staticmethod
    def backward(ctx, gU1, gU2, gV1, gth, gW1, gW2):
        U1, U2, V1, th = ctx.saved_tensors
        if ctx.rank < U1.shape[0]:
            raise NotImplementedError("CSD backward needs a full-rank input")
        gA1, gA2 = csd_backward(U1, U2, V1, th, gth, gW1, gW2)
        return gA1, gA2


def pack_ragged(mats):
    """List of (n_k, n_k) float64 device tensors -> (packed column-major buffer, sizes, offsets)."""
    sizes = [int(M.shape[0]) for M in mats]
    offs, o = [], 0
    for n in sizes:
        offs.append(o)
        o += n * n
    buf = torch.cat([_colmajor(M, "A").reshape(-1) for M in mats]) if mats else None
    return buf, sizes, offs


def unpack_ragged(buf, sizes, offs):
    return [buf[o:o + n * n].view(n, n).t() for n, o in zip(sizes, offs)]


def csd_batched_packed(a1, a2, sizes, offs, rank_mode="auto", **opts):
    """Batched CSD on packed ragged column-major device buffers (see zcsd_dcsd_batched).

    Returns (U1, U2, V1, theta, ranks, info) as packed buffers; theta of problem k
    starts at sum(sizes[:k]).
    """
    bs = len(sizes)
    U1 = torch.empty_like(a1)
    U2 = torch.empty_like(a1)
    V1 = torch.empty_like(a1)
    th = torch.empty(sum(sizes), dtype=torch.float64, device=a1.device)
    nh = (C.c_int * bs)(*sizes)
    oh = (C.c_longlong * bs)(*offs)
    rk = (C.c_int * bs)()
    o = default_opts(rank_mode=rank_mode, **opts)
    info = Info()
    h = handle(a1.device.index)
    st = _lib().zcsd_dcsd_batched(h, bs, nh, oh, _ptr(a1), _ptr(a2), _ptr(U1), _ptr(U2), _ptr(V1),
                                  _ptr(th), rk, C.byref(o), C.byref(info))
    _check(st, "zcsd_dcsd_batched")
    return U1, U2, V1, th, list(rk), info.as_dict()


def small_batch_workspace(batch, device=None, **opts):
    """Workspace (a uint8 device tensor) for csd_batched_small over `batch`
    problems; also uploads the coefficient table for these options
    (zcsd_small_batch_prepare).  Call it outside any graph capture."""
    h = handle(device)
    o = default_opts(**opts)
    nb = C.c_size_t()
    _check(_lib().zcsd_small_batch_prepare(h, int(batch), C.byref(o), C.byref(nb)), "zcsd_small_batch_prepare")
    dev = torch.cuda.current_device() if device is None else int(device)
    return torch.empty(nb.value, dtype=torch.uint8, device=f"cuda:{dev}")


def csd_batched_small(a1, a2, n, off, toff, U1, U2, V1, theta, status, ws, **opts):
    """Enqueue zcsd_dcsd_batched_small on torch's current stream: every buffer
    is a device tensor the caller made (a1, a2, U1, U2, V1, theta float64; n,
    status int32; off, toff int64; ws from small_batch_workspace), so the call
    can be captured in a torch.cuda.CUDAGraph and replayed.  Nothing is
    synchronised or read back: status[k] tells which problems were written
    (low byte 0)."""
    bs = int(n.numel())
    for t, dt, nm in ((a1, torch.float64, "a1"), (a2, torch.float64, "a2"), (U1, torch.float64, "U1"),
                      (U2, torch.float64, "U2"), (V1, torch.float64, "V1"), (theta, torch.float64, "theta"),
                      (n, torch.int32, "n"), (status, torch.int32, "status"), (off, torch.int64, "off"),
                      (toff, torch.int64, "toff"), (ws, torch.uint8, "ws")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise TypeError(f"{nm} must be a contiguous {dt} device tensor")
    if off.numel() != bs or toff.numel() != bs or status.numel() != bs:
        raise ValueError("n, off, toff and status must have one entry per problem")
    h = handle(a1.device.index)
    o = default_opts(**opts)
    st = _lib().zcsd_dcsd_batched_small(h, bs, _ptr(n), _ptr(off), _ptr(toff), _ptr(a1), _ptr(a2), _ptr(U1),
                                        _ptr(U2), _ptr(V1), _ptr(theta), _ptr(status), _ptr(ws),
                                        ws.numel(), C.byref(o))
    _check(st, "zcsd_dcsd_batched_small")


def csd_batched(A1s, A2s, rank_mode="auto", **opts):
    """Batched CSD of lists of (n_k, n_k) pairs: list of (U1, U2, V1, theta, rank)."""
    if len(A1s) != len(A2s) or not A1s:
        raise ValueError("csd_batched: need equal, non-empty lists")
    for a, b in zip(A1s, A2s):
        if a.shape != b.shape or a.dim() != 2 or a.shape[0] != a.shape[1]:
            raise ValueError("csd_batched: every A1[k], A2[k] must be n_k x n_k")
    a1, sizes, offs = pack_ragged(A1s)
    a2, _, _ = pack_ragged(A2s)
    U1, U2, V1, th, ranks, info = csd_batched_packed(a1, a2, sizes, offs, rank_mode=rank_mode, **opts)
    u1, u2, v1 = unpack_ragged(U1, sizes, offs), unpack_ragged(U2, sizes, offs), unpack_ragged(V1, sizes, offs)
    out, t0 = [], 0
    for k, n in enumerate(sizes):
        out.append((u1[k], u2[k], v1[k], th[t0:t0 + n], ranks[k]))
        t0 += n
    return out
