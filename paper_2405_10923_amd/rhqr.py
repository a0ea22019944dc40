"""Thin ctypes binding of librhqr.so (the C ABI declared in include/rhqr.h).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch tensors provide device memory and the current stream.  Matrices are
column-major: an (r x c) matrix is a tensor of shape (r, c) with stride(0) == 1
and leading dimension stride(1).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librhqr.so")

F64, F32, F16, BF16 = 0, 1, 2, 3
SRHT, GAUSS = 0, 1
SCALE_UNIT_PIVOT, SCALE_SQRT2 = 0, 1
REC_M, REC_RCHOL = 0, 1
RHQR_OK, RHQR_ERR_HIP, RHQR_ERR_WORKSPACE, RHQR_ERR_UNSUPPORTED = 0, -1000, -1001, -1002

_lib = None

_vp, _i32, _i64, _u64, _sz, _dp = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_size_t, C.c_void_p

_SIGS = {
    "rhqr_sketch_create": (C.c_int, [C.c_int, _i64, _i32, _i32, _u64, _vp, _i64, _vp, C.POINTER(_vp)]),
    "rhqr_sketch_destroy": (C.c_int, [_vp]),
    "rhqr_sketch_get": (C.c_int, [_vp, _vp, _vp, _vp]),
    "rhqr_sketch_info": (C.c_int, [_vp, C.POINTER(_i64), C.POINTER(_i32), C.POINTER(_i32),
                                   C.POINTER(_i64), C.POINTER(_i32)]),
    "rhqr_sketch_workspace_size": (_sz, [_vp, _i32]),
    "rhqr_sketch": (C.c_int, [_vp, C.c_int, _i64, _i32, _vp, _i64, _vp, _i64, _vp, _sz, _vp]),
    "rhqr_factor_workspace_size": (_sz, [_vp, C.c_int, _i32]),
    "rhqr_factor": (C.c_int, [_vp, C.c_int, _i64, _i32, _vp, _i64, _vp, _i64, _vp, _i64, _vp,
                              _i64, _vp, _i64, C.c_int, _vp, _sz, _vp]),
    "rhqr_factor_noalloc": (C.c_int, [_vp, C.c_int, _i64, _i32, _vp, _i64, _vp, _i64, _vp, _i64,
                                      _vp, _i64, _vp, _i64, C.c_int, _vp, _vp]),
    "rhqr_status": (C.c_int, [_vp, _vp, C.POINTER(_i32)]),
    "rhqr_rgs_workspace_size": (_sz, [_vp, C.c_int, _i32]),
    "rhqr_rgs_factor": (C.c_int, [_vp, C.c_int, _i64, _i32, _vp, _i64, _vp, _i64, _vp, _i64, _vp,
                                  _i64, _vp, _i64, C.c_int, _vp, _sz, _vp]),
    "recrhqr_workspace_size": (_sz, [_vp, C.c_int, _i32]),
    "recrhqr_factor": (C.c_int, [_vp, C.c_int, _i64, _i32, _vp, _i64, _vp, _i64, _vp, _i64, _vp,
                                 _i64, _vp, _i64, _vp, _i64, C.c_int, _vp, _sz, _vp]),
    "rhqr_arnoldi_create": (C.c_int, [_vp, C.c_int, _i64, _i32, _vp, C.POINTER(_vp)]),
    "rhqr_arnoldi_destroy": (C.c_int, [_vp]),
    "rhqr_arnoldi_start": (C.c_int, [_vp, _vp, _vp, C.POINTER(C.c_double), _vp]),
    "rhqr_arnoldi_step": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "rhqr_arnoldi_solution": (C.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "rhqr_arnoldi_basis": (C.c_int, [_vp, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp)]),
    "rhqr_arnoldi_solve_ls": (C.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "rhqr_gmres_csr": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, C.c_double, _i32, _vp,
                                 C.POINTER(_i32), C.POINTER(_i64), _vp]),
    "rhqr_spmv_csr": (C.c_int, [C.c_int, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rhqr_batch_workspace_size": (_sz, [_vp, _i32, C.c_int]),
    "rhqr_batch_create": (C.c_int, [_vp, _i32, C.c_int, C.c_int, _vp, _sz, _vp, C.POINTER(_vp)]),
    "rhqr_batch_factor": (C.c_int, [_vp, C.c_int, _vp]),
    "rhqr_batch_thin_q": (C.c_int, [_vp, _vp, _vp, _vp]),
    "rhqr_batch_status": (C.c_int, [_vp, _vp, _vp]),
    "rhqr_batch_destroy": (C.c_int, [_vp]),
    "rhqr_trim_workspace_size": (_sz, [_vp, C.c_int, _i32]),
    "rhqr_trim_factor": (C.c_int, [_vp, C.c_int, _i64, _i32, _vp, _i64, _vp, _i64, _vp, _i64, _vp,
                                   _i64, _vp, _i64, _vp, _i64, C.c_int, _vp, _sz, _vp]),
    "rhqr_colscale": (C.c_int, [C.c_int, _i64, _i32, _vp, _i64, _vp, _i64, _vp, _vp]),
    "rhqr_scale_r": (C.c_int, [_i32, _vp, _i64, _vp, _vp]),
    "rhqr_profile_begin": (C.c_int, []),
    "rhqr_profile_end": (C.c_int, [_i32, _vp, _vp]),
}


def lib():
    """Load librhqr.so.  Fails loudly when the library has not been built:
    there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build it with "
                               "`python -m paper_2405_10923_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _lib = L
    return _lib


class RHQRError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise RHQRError(f"{what} failed with code {rc}")


def _torch():
    import torch
    return torch


def dtype_code(t):
    torch = _torch()
    return {torch.float64: F64, torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}[t]


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ld(t):
    if t.dim() != 2 or (t.stride(0) != 1 and t.shape[0] > 1):
        raise ValueError("expected a column-major matrix (stride(0) == 1)")
    if t.shape[1] == 1:
        return max(t.shape[0], 1)
    return t.stride(1)


def colmajor_empty(rows, cols, dtype, device):
    torch = _torch()
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def to_colmajor(t):
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    if t.stride(0) == 1 or t.shape[0] == 1:
        return t
    return t.t().contiguous().t()


def workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


class Sketch:
    """Psi = [I_m 0; 0 Omega] for n-row problems (Sec. 2.3, eq. psi)."""

    def __init__(self, kind, n, m, l, seed=0, omega=None):
        torch = _torch()
        self.kind, self.n, self.m, self.l, self.seed = kind, int(n), int(m), int(l), int(seed)
        h = C.c_void_p()
        om = _ptr(omega) if omega is not None else C.c_void_p(0)
        ldo = _ld(omega) if omega is not None else 0
        rc = lib().rhqr_sketch_create(int(kind), self.n, self.m, self.l, C.c_uint64(self.seed), om,
                                      ldo, _stream(), C.byref(h))
        _check(rc, "rhqr_sketch_create")
        self.h = h
        N = C.c_int64()
        lib().rhqr_sketch_info(h, None, None, None, C.byref(N), None)
        self.N = N.value
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "h", None):
            lib().rhqr_sketch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def rows_out(self):
        return self.l + self.m

    def signs_words(self):
        w = np.zeros((self.N + 63) // 64, dtype=np.uint64)
        _check(lib().rhqr_sketch_get(self.h, w.ctypes.data_as(C.c_void_p), None, None), "get")
        return w

    def rows(self):
        r = np.zeros(self.l, dtype=np.int32)
        _check(lib().rhqr_sketch_get(self.h, None, r.ctypes.data_as(C.c_void_p), None), "get")
        return r

    def omega(self):
        o = np.zeros((self.n - self.m) * self.l, dtype=np.float64)
        _check(lib().rhqr_sketch_get(self.h, None, None, o.ctypes.data_as(C.c_void_p)), "get")
        return o.reshape(self.n - self.m, self.l).T


def sketch(sk, X, Y=None, ws=None):
    """Y = Psi X (RHSketch, Alg. 1); X column-major (n x k) on the GPU."""
    X = to_colmajor(X)
    n, k = X.shape
    if Y is None:
        Y = colmajor_empty(sk.rows_out, k, _torch().float64, X.device)
    nb = lib().rhqr_sketch_workspace_size(sk.h, k)
    if ws is None:
        ws = workspace(nb, X.device)
    rc = lib().rhqr_sketch(sk.h, dtype_code(X.dtype), n, k, _ptr(X), _ld(X), _ptr(Y), _ld(Y),
                           _ptr(ws), ws.numel(), _stream())
    _check(rc, "rhqr_sketch")
    return Y


class FactorBuffers:
    """Outputs and workspace of rhqr_factor for one (sketch, dtype, m)."""

    def __init__(self, sk, dtype, m, want_q=False, n=None):
        torch = _torch()
        dev = sk.device
        L = sk.rows_out
        self.S = colmajor_empty(L, m, torch.float64, dev)
        self.T = colmajor_empty(m, m, torch.float64, dev)
        self.R = colmajor_empty(m, m, torch.float64, dev)
        self.Q = colmajor_empty(sk.n, m, dtype, dev) if want_q else None
        self.ws = workspace(lib().rhqr_factor_workspace_size(sk.h, dtype_code(dtype), m), dev)


def factor(sk, W, scaling=SCALE_UNIT_PIVOT, want_q=False, bufs=None, panel=0, outer=0, tpw=0,
           right=False):
    """Left-looking RHQR (Alg. 4).  W (n x m, column-major, GPU) is overwritten
    by U.  ``panel`` >= 2 selects the blocked schedule (panels of that many
    columns); ``outer`` > panel groups the panels in outer panels of that many
    columns (two levels); ``panel=None`` takes the autotuned schedule of the
    problem's size (schedules.lookup); ``tpw`` sets the transform tiles per
    workgroup of the refresh pass (0: the library's choice).  ``right=True``
    runs right-looking RHQR (Alg. 3) instead (the schedule arguments must then
    be 0).  Returns dict(U=W, S, T, R, Q)."""
    n, m = W.shape
    if right:
        if panel or outer or tpw:
            raise ValueError("right-looking RHQR takes no schedule options")
    elif panel is None:
        from .schedules import lookup
        panel, outer, tpw, _ = lookup(W.dtype, n, m)
    if bufs is None:
        bufs = FactorBuffers(sk, W.dtype, m, want_q)
    Q = bufs.Q if want_q else None
    rc = lib().rhqr_factor(sk.h, dtype_code(W.dtype), n, m, _ptr(W), _ld(W), _ptr(bufs.S),
                           _ld(bufs.S), _ptr(bufs.T), _ld(bufs.T), _ptr(bufs.R), _ld(bufs.R),
                           _ptr(Q), _ld(Q) if Q is not None else 0,
                           int(scaling) | (int(panel) << 8) | (int(outer) << 16) | (int(tpw) << 24)
                           | ((1 << 29) if right else 0),
                           _ptr(bufs.ws),
                           bufs.ws.numel(), _stream())
    _check(rc, "rhqr_factor")
    return dict(U=W, S=bufs.S, T=bufs.T, R=bufs.R, Q=Q, ws=bufs.ws)


def rgs(sk, W, panel=0, outer=0):
    """BLAS2-RGS (Alg. 9) by rhqr_rgs_factor.  ``sk`` has n + m rows and head
    m; W (n x m, column-major, GPU) is read only.  Returns dict(Q (n x m view
    of the (n+m)-row output), S, T, R, ws)."""
    torch = _torch()
    n, m = W.shape
    dev = W.device
    Qb = colmajor_empty(n + m, m, W.dtype, dev)
    S = colmajor_empty(sk.rows_out, m, torch.float64, dev)
    T = colmajor_empty(m, m, torch.float64, dev)
    R = colmajor_empty(m, m, torch.float64, dev)
    ws = workspace(lib().rhqr_rgs_workspace_size(sk.h, dtype_code(W.dtype), m), dev)
    rc = lib().rhqr_rgs_factor(sk.h, dtype_code(W.dtype), n, m, _ptr(W), _ld(W), _ptr(Qb), _ld(Qb),
                               _ptr(S), _ld(S), _ptr(T), _ld(T), _ptr(R), _ld(R),
                               (int(panel) << 8) | (int(outer) << 16), _ptr(ws), ws.numel(),
                               _stream())
    _check(rc, "rhqr_rgs_factor")
    return dict(Q=Qb[m:], Qfull=Qb, S=S, T=T, R=R, ws=ws)


def trim(sk, W, scaling=SCALE_UNIT_PIVOT, want_q=True):
    """Left-looking trimRHQR (Alg. 12) by rhqr_trim_factor.  ``sk`` is an SRHT
    sketch with head 0 (Omega on every row: Sketch(SRHT, n, 0, l)); W (n x m,
    column-major, GPU, float64 or float32) is overwritten by U.  Returns
    dict(U, S = Omega U, T, Tt, R, Q, ws)."""
    torch = _torch()
    n, m = W.shape
    dev = W.device
    S = colmajor_empty(sk.l, m, torch.float64, dev)
    T = colmajor_empty(m, m, torch.float64, dev)
    Tt = colmajor_empty(m, m, torch.float64, dev)
    R = colmajor_empty(m, m, torch.float64, dev)
    Q = colmajor_empty(n, m, W.dtype, dev) if want_q else None
    ws = workspace(lib().rhqr_trim_workspace_size(sk.h, dtype_code(W.dtype), m), dev)
    rc = lib().rhqr_trim_factor(sk.h, dtype_code(W.dtype), n, m, _ptr(W), _ld(W), _ptr(S), sk.l,
                                _ptr(T), _ld(T), _ptr(Tt), _ld(Tt), _ptr(R), _ld(R), _ptr(Q),
                                _ld(Q) if Q is not None else 0, int(scaling), _ptr(ws), ws.numel(),
                                _stream())
    _check(rc, "rhqr_trim_factor")
    return dict(U=W, S=S, T=T, Tt=Tt, R=R, Q=Q, ws=ws)


def colscale(W64, dtype, out=None, scale=None):
    """Unit max-norm column scaling of a float64 W (n x m, column-major, GPU)
    rounded to ``dtype`` (rhqr_colscale).  Returns (W D^-1 in dtype, d)."""
    torch = _torch()
    n, m = W64.shape
    if out is None:
        out = colmajor_empty(n, m, dtype, W64.device)
    if scale is None:
        scale = torch.empty(m, dtype=torch.float64, device=W64.device)
    rc = lib().rhqr_colscale(dtype_code(dtype), n, m, _ptr(W64), _ld(W64), _ptr(out), _ld(out),
                             _ptr(scale), _stream())
    _check(rc, "rhqr_colscale")
    return out, scale


def scale_r(R, scale):
    """R <- R D in place (rhqr_scale_r)."""
    m = R.shape[0]
    _check(lib().rhqr_scale_r(m, _ptr(R), _ld(R), _ptr(scale), _stream()), "rhqr_scale_r")
    return R


def status(ws):
    info = C.c_int32()
    _check(lib().rhqr_status(_ptr(ws), _stream(), C.byref(info)), "rhqr_status")
    return info.value


def recrhqr(sk, W, mode=REC_M, want_q=True):
    """recRHQR (Alg. 6).  W is read only.  Returns dict(U, S, T, R, Q)."""
    torch = _torch()
    n, m = W.shape
    dev = W.device
    L = sk.rows_out
    S = colmajor_empty(L, m, torch.float64, dev)
    T = colmajor_empty(m, m, torch.float64, dev)
    R = colmajor_empty(m, m, torch.float64, dev)
    U = colmajor_empty(n, m, W.dtype, dev) if mode == REC_M else None
    Q = colmajor_empty(n, m, W.dtype, dev) if want_q else None
    ws = workspace(lib().recrhqr_workspace_size(sk.h, dtype_code(W.dtype), m), dev)
    rc = lib().recrhqr_factor(sk.h, dtype_code(W.dtype), n, m, _ptr(W), _ld(W), _ptr(U),
                              _ld(U) if U is not None else 0, _ptr(S), _ld(S), _ptr(T), _ld(T),
                              _ptr(R), _ld(R), _ptr(Q), _ld(Q) if Q is not None else 0, int(mode),
                              _ptr(ws), ws.numel(), _stream())
    _check(rc, "recrhqr_factor")
    return dict(U=U, S=S, T=T, R=R, Q=Q, ws=ws)


class _Problem(C.Structure):
    _fields_ = [("sketch", _vp), ("d_W", _vp), ("ldw", _i64), ("d_S", _vp), ("lds", _i64),
                ("d_T", _vp), ("ldt", _i64), ("d_R", _vp), ("ldr", _i64)]


class Batch:
    """Batched left-looking RHQR (rhqr_batch_*): ``problems`` is a list of
    (Sketch, W) pairs, W (n x m, column-major, GPU, one dtype for the batch)
    overwritten by U.  Allocates S, T, R per problem and the batch workspace;
    ``panel`` >= 2 selects the blocked schedule (0: column by column) and
    ``outer`` > panel groups its panels in outer panels (as in ``factor``);
    ``factor(graph)`` runs the whole batch (as a replayed hipGraph when
    ``graph`` is true), ``thin_q()`` forms every problem's thin Q afterwards.
    ``outputs[i]`` = dict(U, S, T, R[, Q]) in caller order."""

    def __init__(self, problems, scaling=SCALE_UNIT_PIVOT, panel=0, outer=0):
        torch = _torch()
        self._lib = lib()
        self.problems = list(problems)
        dt = self.problems[0][1].dtype
        self.dtype = dt
        arr = (_Problem * len(self.problems))()
        self.outputs = []
        for i, (sk, W) in enumerate(self.problems):
            n, m = W.shape
            if W.dtype != dt or n != sk.n or m != sk.m:
                raise ValueError(f"problem {i}: W does not match its sketch or the batch dtype")
            dev = W.device
            S = colmajor_empty(sk.rows_out, m, torch.float64, dev)
            T = colmajor_empty(m, m, torch.float64, dev)
            R = colmajor_empty(m, m, torch.float64, dev)
            self.outputs.append(dict(U=W, S=S, T=T, R=R))
            arr[i] = _Problem(sk.h.value, W.data_ptr(), _ld(W), S.data_ptr(), _ld(S), T.data_ptr(),
                              _ld(T), R.data_ptr(), _ld(R))
        self._arr = arr
        code = dtype_code(dt)
        nb = self._lib.rhqr_batch_workspace_size(arr, len(arr), code)
        if nb == 0:
            raise RHQRError("rhqr_batch_workspace_size rejected the problems")
        self.ws = workspace(nb, self.problems[0][1].device)
        h = C.c_void_p()
        _check(self._lib.rhqr_batch_create(arr, len(arr), code,
                                           int(scaling) | (int(panel) << 8) | (int(outer) << 16),
                                           _ptr(self.ws),
                                           self.ws.numel(), _stream(), C.byref(h)),
               "rhqr_batch_create")
        self.h = h

    def factor(self, graph=False):
        _check(self._lib.rhqr_batch_factor(self.h, 1 if graph else 0, _stream()),
               "rhqr_batch_factor")
        return self.outputs

    def thin_q(self, Qs=None):
        """Thin Q of every problem (rhqr_batch_thin_q) after factor(): into
        ``Qs[i]`` (n x m, column-major, the batch dtype; allocated when None);
        returns the list in caller order."""
        if Qs is None:
            Qs = [colmajor_empty(W.shape[0], W.shape[1], self.dtype, W.device)
                  for _, W in self.problems]
        k = len(self.problems)
        ptrs = (C.c_void_p * k)(*[Q.data_ptr() for Q in Qs])
        lds = (C.c_int64 * k)(*[_ld(Q) for Q in Qs])
        _check(self._lib.rhqr_batch_thin_q(self.h, ptrs, lds, _stream()), "rhqr_batch_thin_q")
        for out, Q in zip(self.outputs, Qs):
            out["Q"] = Q
        return Qs

    def status(self):
        info = (C.c_int32 * len(self.problems))()
        _check(self._lib.rhqr_batch_status(self.h, _stream(), info), "rhqr_batch_status")
        return list(info)

    def close(self):
        if getattr(self, "h", None):
            self._lib.rhqr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_begin():
    _check(lib().rhqr_profile_begin(), "rhqr_profile_begin")


# kernel classes of rhqr_profile_end, in the order of RHQR_PROF_*
PROF_CLASSES = ("tall", "panel_mx", "panel_valu", "presketch", "red", "fin", "qtail", "trsm",
                "hqr", "right_vec", "right_apply")


def profile_end():
    """Summed kernel time (ms) and launch count per kernel class since
    profile_begin(), from HIP events recorded by each dispatch:
    {class name: (ms, launches)}."""
    k = len(PROF_CLASSES)
    ms = (C.c_double * k)()
    cnt = (C.c_int64 * k)()
    _check(lib().rhqr_profile_end(k, ms, cnt), "rhqr_profile_end")
    return {name: (ms[i], cnt[i]) for i, name in enumerate(PROF_CLASSES)}


class CSR:
    """A float64 CSR matrix on the GPU (row pointers int64, indices int32)."""

    def __init__(self, indptr, indices, values, n, device=None):
        torch = _torch()
        dev = device or torch.device("cuda", torch.cuda.current_device())
        self.n = int(n)
        self.ptr = torch.as_tensor(np.asarray(indptr, dtype=np.int64), device=dev)
        self.idx = torch.as_tensor(np.asarray(indices, dtype=np.int32), device=dev)
        self.val = torch.as_tensor(np.asarray(values, dtype=np.float64), device=dev)

    def matvec(self, x, y=None):
        torch = _torch()
        if y is None:
            y = torch.empty_like(x)
        rc = lib().rhqr_spmv_csr(dtype_code(x.dtype), self.n, _ptr(self.ptr), _ptr(self.idx),
                                 _ptr(self.val), _ptr(x), _ptr(y), _stream())
        _check(rc, "rhqr_spmv_csr")
        return y


class Arnoldi:
    """RHQR-Arnoldi (Alg. 7) state: up to ``mmax`` steps; the sketch must have
    head m = mmax + 1."""

    def __init__(self, sk, dtype, mmax):
        h = C.c_void_p()
        rc = lib().rhqr_arnoldi_create(sk.h, dtype_code(dtype), sk.n, int(mmax), _stream(),
                                       C.byref(h))
        _check(rc, "rhqr_arnoldi_create")
        self.h, self.sk, self.dtype, self.mmax = h, sk, dtype, int(mmax)

    def close(self):
        if getattr(self, "h", None):
            lib().rhqr_arnoldi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def start(self, r0, q1):
        beta = C.c_double()
        _check(lib().rhqr_arnoldi_start(self.h, _ptr(r0), _ptr(q1), C.byref(beta), _stream()),
               "rhqr_arnoldi_start")
        return beta.value

    def step(self, w, qnext, hcol):
        _check(lib().rhqr_arnoldi_step(self.h, _ptr(w), _ptr(qnext), _ptr(hcol), _stream()),
               "rhqr_arnoldi_step")

    def solution(self, j, y, x):
        _check(lib().rhqr_arnoldi_solution(self.h, int(j), _ptr(y), _ptr(x), _stream()),
               "rhqr_arnoldi_solution")

    def solve_ls(self, j, y, res=None):
        """y (j float64, GPU) <- argmin ||beta e_1 - H_{j+1,j} y|| (rhqr_arnoldi_solve_ls)."""
        _check(lib().rhqr_arnoldi_solve_ls(self.h, int(j), _ptr(y), _ptr(res), _stream()),
               "rhqr_arnoldi_solve_ls")


def gmres(A, b, sk, m, dtype, tol=1e-6, max_cycles=1000, x0=None):
    """Restarted RHQR-GMRES(m) (Alg. 8) by rhqr_gmres_csr: Krylov basis in
    ``dtype``, Hessenberg least squares and solution update in float64, true
    residual recomputed in float64 after every cycle, all in the library.
    ``A`` is a CSR, ``b`` a float64 GPU vector.  Returns (x float64, list of
    relative residuals after each cycle, total Arnoldi steps)."""
    torch = _torch()
    x = torch.zeros(A.n, dtype=torch.float64, device=b.device) if x0 is None else x0.clone()
    arn = Arnoldi(sk, dtype, m)
    hist = np.zeros(max_cycles, dtype=np.float64)
    cyc, steps = C.c_int32(), C.c_int64()
    rc = lib().rhqr_gmres_csr(arn.h, _ptr(A.ptr), _ptr(A.idx), _ptr(A.val), _ptr(b), _ptr(x),
                              float(tol), int(max_cycles), hist.ctypes.data_as(C.c_void_p),
                              C.byref(cyc), C.byref(steps), _stream())
    arn.close()
    _check(rc, "rhqr_gmres_csr")
    return x, [float(v) for v in hist[:cyc.value]], steps.value
