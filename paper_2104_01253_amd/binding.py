"""Thin ctypes binding of libdcgs2.so (argument marshalling only).

Every step of the expansion runs in the HIP library; this module only turns
torch device tensors into pointers, sizes and the context's stream, and the
library's status codes into Python values.  Column-major matrices are torch
tensors of shape (m, ncols) with stride (1, ld) -- see ``colmajor_empty``.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdcgs2.so")

OK, EINVAL, EDEVICE, ENOMEM = 0, -1, -2, -3
BREAKDOWN, NOT_CONVERGED, NONFINITE = 1, 2, 3
OP_CSR, OP_STENCIL5, OP_STENCIL7 = 0, 1, 2
MAX_N = 1024

EXPORTS = ("dcgs2_create", "dcgs2_destroy", "dcgs2_set_tolerances", "dcgs2_qr", "dcgs2_arnoldi",
           "gmres_solve", "krylov_schur_eigs", "dcgs2_apply", "dcgs2_status_str",
           "dcgs2_profile_enable", "dcgs2_profile_read", "dcgs2_set_qr_schedule",
           "dcgs2_qr_q32", "dcgs2_arnoldi_q32", "dcgs2_set_basis_precision", "cgs2_qr",
           "dcgs2_set_tuning", "dcgs2_get_tuning", "krylov_schur_batched",
           "dcgs2_mlp_create", "dcgs2_mlp_destroy", "dcgs2_mlp_num_params",
           "dcgs2_mlp_set_params", "dcgs2_mlp_get_params", "dcgs2_mlp_get_grads",
           "dcgs2_mlp_forward", "dcgs2_mlp_loss_grad", "dcgs2_mlp_adam",
           "dcgs2_guess_features", "dcgs2_guess_targets", "dcgs2_guess_prolong",
           "dcgs2_guess_guard", "mgs_qr", "dcgs2_arnoldi_steps", "dcgs2_qr_steps",
           "dcgs2_qr_noalloc", "dcgs2_arnoldi_batched",
           "gmres_batched")
(TUNE_FUSED_WAVES, TUNE_REDUCE_GRID, TUNE_FUSED_MIN_J, TUNE_BATCH_REDUCE_ROWS,
 TUNE_FUSED_PAIR_SLOTS, TUNE_BATCH_DENSE, TUNE_MATVEC_FOLD, TUNE_UPDATE_GRID) = range(8)


class Stats(ctypes.Structure):
    _fields_ = [("reductions", c_int32), ("pyth_fallbacks", c_int32),
                ("breakdown_step", c_int32), ("kernels", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Op(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("m", c_int64), ("rowptr", c_void_p), ("colind", c_void_p),
                ("val", c_void_p), ("nnz", c_int64), ("nx", c_int32), ("ny", c_int32),
                ("nz", c_int32), ("c0", c_double), ("cxm", c_double), ("cxp", c_double),
                ("cym", c_double), ("cyp", c_double), ("czm", c_double), ("czp", c_double)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", c_int64), ("total_ms", c_double),
                ("bytes", c_double)]


class GmresInfo(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("cycles", c_int32), ("status", c_int32), ("pad", c_int32),
                ("relres_true", c_double), ("relres_est", c_double), ("st", Stats)]


class KsInfo(ctypes.Structure):
    _fields_ = [("restarts", c_int32), ("nconv", c_int32), ("matvecs", c_int32),
                ("status", c_int32), ("resid", c_double), ("st", Stats)]


class Stencil2d(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("c0", c_double), ("cxm", c_double),
                ("cxp", c_double), ("cym", c_double), ("cyp", c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libdcgs2.so; raises if it is not built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2104_01253_amd.build`")
    lib = ctypes.CDLL(path)
    lib.dcgs2_create.argtypes = [POINTER(c_void_p), c_int, c_void_p]
    lib.dcgs2_destroy.argtypes = [c_void_p]
    lib.dcgs2_set_tolerances.argtypes = [c_void_p, c_double, c_double]
    lib.dcgs2_qr.argtypes = [c_void_p, c_int64, c_int32, c_void_p, c_int64, c_void_p, c_int64,
                             c_void_p, c_int32, POINTER(Stats)]
    lib.dcgs2_arnoldi.argtypes = [c_void_p, POINTER(Op), c_void_p, c_int32, c_void_p, c_int64,
                                  c_void_p, c_int32, POINTER(Stats)]
    lib.gmres_solve.argtypes = [c_void_p, POINTER(Op), c_void_p, c_void_p, c_int32, c_double,
                                c_int32, POINTER(GmresInfo)]
    lib.krylov_schur_eigs.argtypes = [c_void_p, POINTER(Op), c_int32, c_int32, c_int32, c_double,
                                      c_int32, c_void_p, c_void_p, c_void_p, POINTER(KsInfo)]
    lib.krylov_schur_batched.argtypes = [c_void_p, c_int32, POINTER(Stencil2d), c_int32, c_int32,
                                         c_int32, c_double, c_int32, c_void_p, c_void_p,
                                         c_void_p, POINTER(KsInfo), c_int32]
    lib.dcgs2_apply.argtypes = [c_void_p, POINTER(Op), c_void_p, c_void_p]
    lib.gmres_batched.argtypes = [c_void_p, c_int32, POINTER(Stencil2d), c_void_p, c_void_p,
                                  c_void_p, c_double, c_int32, POINTER(GmresInfo)]
    lib.dcgs2_arnoldi_batched.argtypes = [c_void_p, c_int32, POINTER(Stencil2d), c_void_p,
                                          c_void_p, c_void_p, c_void_p, c_void_p,
                                          POINTER(Stats)]
    lib.dcgs2_arnoldi_steps.argtypes = [c_void_p, POINTER(Op), c_int32, c_int32, c_void_p,
                                        c_int64, c_void_p, c_void_p, c_void_p, c_int32, c_double,
                                        c_void_p, POINTER(Stats)]
    lib.dcgs2_qr_steps.argtypes = [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_int64,
                                   c_void_p, c_int64, c_void_p, c_void_p, c_int32, c_void_p,
                                   c_double, c_void_p, POINTER(Stats)]
    lib.dcgs2_profile_enable.argtypes = [c_void_p, c_int]
    lib.dcgs2_set_qr_schedule.argtypes = [c_void_p, c_int]
    lib.dcgs2_set_basis_precision.argtypes = [c_void_p, c_int]
    lib.dcgs2_qr_q32.argtypes = lib.dcgs2_qr.argtypes
    lib.cgs2_qr.argtypes = lib.dcgs2_qr.argtypes
    lib.mgs_qr.argtypes = lib.dcgs2_qr.argtypes
    lib.dcgs2_qr_noalloc.argtypes = lib.dcgs2_qr.argtypes
    lib.dcgs2_set_tuning.argtypes = [c_void_p, c_int32, c_int32]
    lib.dcgs2_get_tuning.argtypes = [c_void_p, c_int32, POINTER(c_int32)]
    lib.dcgs2_arnoldi_q32.argtypes = lib.dcgs2_arnoldi.argtypes
    lib.dcgs2_profile_read.argtypes = [c_void_p, POINTER(KernelStat), c_int32, c_int32]
    lib.dcgs2_status_str.argtypes = [c_int]
    lib.dcgs2_status_str.restype = ctypes.c_char_p
    c_i32p = POINTER(c_int32)
    lib.dcgs2_mlp_create.argtypes = [c_void_p, c_int32, c_i32p, c_int32, POINTER(c_void_p)]
    lib.dcgs2_mlp_destroy.argtypes = [c_void_p]
    lib.dcgs2_mlp_num_params.argtypes = [c_void_p, POINTER(c_int64)]
    lib.dcgs2_mlp_set_params.argtypes = [c_void_p, c_void_p]
    lib.dcgs2_mlp_get_params.argtypes = [c_void_p, c_void_p]
    lib.dcgs2_mlp_get_grads.argtypes = [c_void_p, c_void_p]
    lib.dcgs2_mlp_forward.argtypes = [c_void_p, c_int32, c_void_p, c_void_p]
    lib.dcgs2_mlp_loss_grad.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, POINTER(c_double)]
    lib.dcgs2_mlp_adam.argtypes = [c_void_p, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float]
    lib.dcgs2_guess_features.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                         c_int32, c_int32, c_void_p, c_void_p]
    lib.dcgs2_guess_targets.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                        c_double, c_void_p]
    lib.dcgs2_guess_prolong.argtypes = lib.dcgs2_guess_targets.argtypes
    lib.dcgs2_guess_guard.argtypes = [c_void_p, POINTER(Op), c_void_p, c_void_p, c_double,
                                      c_i32p, POINTER(c_double)]
    for name in EXPORTS:
        if name != "dcgs2_status_str":
            getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def status_str(code: int) -> str:
    return load().dcgs2_status_str(code).decode()


class DCGS2Error(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {status_str(code)} ({code})")
        self.code = code


# ---- tensors ----------------------------------------------------------------------
def colmajor_empty(m: int, ncols: int, ld: int | None = None, device="cuda", dtype=None):
    """Uninitialised column-major m x ncols device matrix with leading dimension ld."""
    import torch
    ld = ((m + 63) // 64) * 64 if ld is None else ld
    buf = torch.empty((ncols, ld), dtype=dtype or torch.float64, device=device)
    return buf.t()[:m]


def colmajor_from_numpy(A: np.ndarray, device="cuda", ld: int | None = None):
    import torch
    m, n = A.shape
    out = colmajor_empty(m, n, ld, device)
    out.copy_(torch.from_numpy(np.ascontiguousarray(A)).to(device))
    return out


def _colmajor_args(T, name, allow32=False):
    import torch
    ok = (torch.float64, torch.float32) if allow32 else (torch.float64,)
    if T.dim() != 2 or T.dtype not in ok or not T.is_cuda:
        raise ValueError(f"{name}: expected a 2-D {'float32/' if allow32 else ''}float64 CUDA tensor")
    if T.stride(0) != 1:
        raise ValueError(f"{name}: expected column-major layout (stride(0) == 1)")
    ld = T.stride(1) if T.shape[1] > 1 else max(T.shape[0], 1)
    return T.data_ptr(), ld


def _vec_ptr(t, name, m=None):
    if t.dim() != 1 or t.dtype != _f64() or not t.is_cuda or t.stride(0) != 1:
        raise ValueError(f"{name}: expected a contiguous 1-D float64 CUDA tensor")
    if m is not None and t.numel() != m:
        raise ValueError(f"{name}: expected length {m}")
    return t.data_ptr()


def _f64():
    import torch
    return torch.float64


def _ptr(t, dtype):
    """Device pointer of a contiguous CUDA tensor of the given dtype."""
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous CUDA tensor of {dtype}")
    return t.data_ptr()


class MLP:
    """FP32 perceptron on the device (dcgs2_mlp_*): widths[0] -> ... -> widths[-1]."""

    def __init__(self, ctx: "Context", widths, max_batch: int):
        self._lib = ctx._lib
        self.widths = [int(w) for w in widths]
        self.max_batch = int(max_batch)
        arr = (c_int32 * len(self.widths))(*self.widths)
        h = c_void_p()
        rc = self._lib.dcgs2_mlp_create(ctx._h, len(self.widths) - 1, arr, self.max_batch,
                                        ctypes.byref(h))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_mlp_create")
        self._h = h
        n = c_int64()
        self._lib.dcgs2_mlp_num_params(h, ctypes.byref(n))
        self.num_params = n.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.dcgs2_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, layers):
        """[(W (K x N), b (N,)), ...] -> flat float32 parameter vector."""
        return np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(),
                                               np.asarray(b, np.float32).ravel()])
                               for W, b in layers])

    def unpack(self, flat):
        out, o = [], 0
        for K, N in zip(self.widths[:-1], self.widths[1:]):
            W = flat[o:o + K * N].reshape(K, N)
            o += K * N
            out.append((W, flat[o:o + N]))
            o += N
        return out

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        if flat.size != self.num_params:
            raise ValueError("parameter count")
        rc = self._lib.dcgs2_mlp_set_params(self._h, flat.ctypes.data_as(c_void_p))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_mlp_set_params")

    def get_params(self):
        out = np.empty(self.num_params, dtype=np.float32)
        rc = self._lib.dcgs2_mlp_get_params(self._h, out.ctypes.data_as(c_void_p))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_mlp_get_params")
        return out

    def get_grads(self):
        out = np.empty(self.num_params, dtype=np.float32)
        rc = self._lib.dcgs2_mlp_get_grads(self._h, out.ctypes.data_as(c_void_p))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_mlp_get_grads")
        return out

    def forward(self, X, out=None):
        import torch
        Y = out if out is not None else torch.empty((X.shape[0], self.widths[-1]),
                                                    dtype=torch.float32, device=X.device)
        rc = self._lib.dcgs2_mlp_forward(self._h, X.shape[0], _ptr(X, torch.float32),
                                         _ptr(Y, torch.float32))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_mlp_forward")
        return Y

    def loss_grad(self, X, T) -> float:
        import torch
        loss = c_double()
        rc = self._lib.dcgs2_mlp_loss_grad(self._h, X.shape[0], _ptr(X, torch.float32),
                                           _ptr(T, torch.float32), ctypes.byref(loss))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_mlp_loss_grad")
        return loss.value

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        rc = self._lib.dcgs2_mlp_adam(self._h, lr, beta1, beta2, eps)
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_mlp_adam")


# ---- operators --------------------------------------------------------------------
def stencil_coefficients(grid, D=1.0, vel=None, h=None):
    """Central-difference coefficients of -D Lap(u) + v.grad(u) (Dirichlet, h = 1/(n+1))."""
    d = len(grid)
    vel = (0.0,) * d if vel is None else tuple(vel)
    if h is None:
        hs = tuple(1.0 / (n + 1) for n in grid)
    else:
        hs = (float(h),) * d if np.isscalar(h) else tuple(h)
    c0 = 0.0
    lo, hi = [], []
    for n, v, hh in zip(grid, vel, hs):
        dif = D / (hh * hh)
        adv = v / (2.0 * hh)
        c0 += 2.0 * dif
        lo.append(-dif - adv)    # coefficient of the neighbour at i - 1 along this axis
        hi.append(-dif + adv)    # coefficient of the neighbour at i + 1
    while len(lo) < 3:
        lo.append(0.0)
        hi.append(0.0)
    return c0, lo, hi


def stencil_op(grid, D=1.0, vel=None, h=None) -> Op:
    grid = tuple(int(g) for g in grid)
    c0, lo, hi = stencil_coefficients(grid, D, vel, h)
    op = Op()
    op.kind = OP_STENCIL5 if len(grid) == 2 else OP_STENCIL7
    if len(grid) == 1:
        grid = (grid[0], 1)
        op.kind = OP_STENCIL5
    op.m = int(np.prod(grid))
    op.nx, op.ny = grid[0], grid[1]
    op.nz = grid[2] if len(grid) == 3 else 1
    op.c0 = c0
    op.cxm, op.cxp, op.cym, op.cyp, op.czm, op.czp = lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]
    return op


def stencil2d(grid, D=1.0, vel=None, h=None) -> Stencil2d:
    """Batched-solver descriptor of a 2-D convection-diffusion stencil."""
    nx, ny = (int(g) for g in grid)
    c0, lo, hi = stencil_coefficients((nx, ny), D, vel, h)
    d = Stencil2d()
    d.nx, d.ny, d.c0 = nx, ny, c0
    d.cxm, d.cxp, d.cym, d.cyp = lo[0], hi[0], lo[1], hi[1]
    return d


def csr_op(rowptr, colind, val) -> Op:
    """rowptr/colind: int32 CUDA tensors, val: float64 CUDA tensor (kept alive by the caller)."""
    import torch
    if rowptr.dtype != torch.int32 or colind.dtype != torch.int32 or val.dtype != torch.float64:
        raise ValueError("csr_op: rowptr/colind int32, val float64")
    op = Op()
    op.kind = OP_CSR
    op.m = rowptr.numel() - 1
    op.rowptr, op.colind, op.val = rowptr.data_ptr(), colind.data_ptr(), val.data_ptr()
    op.nnz = val.numel()
    return op


def batched_basis_offsets(ops, n):
    """Element offsets of the instance bases in dcgs2_arnoldi_batched's Q, and its size."""
    offs, total = [], 0
    for o, k in zip(ops, n):
        ld = ((o.nx * o.ny + 63) // 64) * 64
        offs.append(total)
        total += ld * (int(k) + 1)
    return offs, total


# ---- context ----------------------------------------------------------------------
class Context:
    """A libdcgs2 context bound to one device and one HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        lib = load()
        handle = c_void_p()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        rc = lib.dcgs2_create(ctypes.byref(handle), device, c_void_p(stream))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_create")
        self._h = handle
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.dcgs2_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_tolerances(self, tau=1e-8, eta=1e-12):
        rc = self._lib.dcgs2_set_tolerances(self._h, tau, eta)
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_set_tolerances")

    # -- entry points -------------------------------------------------------------
    def qr(self, B, Q):
        """DCGS2 QR of column-major B into Q (float64, or float32 for the FP32-stored
        basis); returns (R (numpy n x n), status, stats)."""
        import torch
        m, n = B.shape
        pb, ldb = _colmajor_args(B, "B")
        pq, ldq = _colmajor_args(Q, "Q", allow32=True)
        if Q.shape != (m, n):
            raise ValueError("Q must have B's shape")
        R = np.zeros((n, n), order="F")
        st = Stats()
        fn = self._lib.dcgs2_qr_q32 if Q.dtype == torch.float32 else self._lib.dcgs2_qr
        rc = fn(self._h, m, n, pb, ldb, pq, ldq, R.ctypes.data_as(c_void_p), n, ctypes.byref(st))
        if rc < 0:
            raise DCGS2Error(rc, "dcgs2_qr")
        return R, rc, st.as_dict()

    def qr_noalloc(self, B, Q):
        """dcgs2_qr through the allocation-free entry point (fixed library scratch;
        m <= 2,097,152, n <= 128); returns (R, status, stats)."""
        m, n = B.shape
        pb, ldb = _colmajor_args(B, "B")
        pq, ldq = _colmajor_args(Q, "Q")
        if Q.shape != (m, n):
            raise ValueError("Q must have B's shape")
        R = np.zeros((n, n), order="F")
        st = Stats()
        rc = self._lib.dcgs2_qr_noalloc(self._h, m, n, pb, ldb, pq, ldq,
                                        R.ctypes.data_as(c_void_p), n, ctypes.byref(st))
        if rc < 0:
            raise DCGS2Error(rc, "dcgs2_qr_noalloc", "dcgs2_arnoldi_batched",
           "gmres_batched")
        return R, rc, st.as_dict()

    def cgs2_qr(self, B, Q):
        """Comparator: CGS2 QR (three reductions per column); returns (R, status, stats)."""
        m, n = B.shape
        pb, ldb = _colmajor_args(B, "B")
        pq, ldq = _colmajor_args(Q, "Q")
        if Q.shape != (m, n):
            raise ValueError("Q must have B's shape")
        R = np.zeros((n, n), order="F")
        st = Stats()
        rc = self._lib.cgs2_qr(self._h, m, n, pb, ldb, pq, ldq, R.ctypes.data_as(c_void_p), n,
                               ctypes.byref(st))
        if rc < 0:
            raise DCGS2Error(rc, "cgs2_qr")
        return R, rc, st.as_dict()

    def mgs_qr(self, B, Q):
        """Comparator: column-by-column MGS QR (n(n+1)/2 reductions); (R, status, stats)."""
        m, n = B.shape
        pb, ldb = _colmajor_args(B, "B")
        pq, ldq = _colmajor_args(Q, "Q")
        if Q.shape != (m, n):
            raise ValueError("Q must have B's shape")
        R = np.zeros((n, n), order="F")
        st = Stats()
        rc = self._lib.mgs_qr(self._h, m, n, pb, ldb, pq, ldq, R.ctypes.data_as(c_void_p), n,
                              ctypes.byref(st))
        if rc < 0:
            raise DCGS2Error(rc, "mgs_qr")
        return R, rc, st.as_dict()

    def arnoldi(self, op: Op, r0, n: int, Q):
        """n DCGS2 Arnoldi steps from r0 into Q (m x (n+1)); returns (H, status, stats)."""
        import torch
        pr = _vec_ptr(r0, "r0", op.m)
        pq, ldq = _colmajor_args(Q, "Q", allow32=True)
        if Q.shape[0] != op.m or Q.shape[1] < n + 1:
            raise ValueError("Q must be m x (n+1)")
        H = np.zeros((n + 1, n), order="F")
        st = Stats()
        fn = self._lib.dcgs2_arnoldi_q32 if Q.dtype == torch.float32 else self._lib.dcgs2_arnoldi
        rc = fn(self._h, ctypes.byref(op), pr, n, pq, ldq, H.ctypes.data_as(c_void_p), n + 1,
                ctypes.byref(st))
        if rc < 0:
            raise DCGS2Error(rc, "dcgs2_arnoldi")
        return H, rc, st.as_dict()

    def arnoldi_steps(self, op: Op, j0: int, j1: int, Q, w, H, K, rho: float, record=True):
        """Steps j0..j1 of Alg. arnoldi from the state (Q columns, w, H, K, rho); Q and w
        (device) and H, K (numpy float64, Fortran order, >= j1 rows, >= j1-1 columns) are
        updated in place.  Returns (records (j1-j0+1, 3 j1 + 1) or None, status, stats)."""
        pq, ldq = _colmajor_args(Q, "Q")
        pw = _vec_ptr(w, "w", op.m)
        for name, M in (("H", H), ("K", K)):
            if (M.dtype != np.float64 or not M.flags.f_contiguous or M.shape[0] < j1
                    or M.shape[1] < j1 - 1):
                raise ValueError(f"{name} must be a Fortran float64 array of >= j1 x (j1-1)")
        if H.shape[0] != K.shape[0]:
            raise ValueError("H and K need the same leading dimension")
        rec = np.empty((j1 - j0 + 1, 3 * j1 + 1)) if record else None
        st = Stats()
        rc = self._lib.dcgs2_arnoldi_steps(
            self._h, ctypes.byref(op), j0, j1, pq, ldq, pw, H.ctypes.data_as(c_void_p),
            K.ctypes.data_as(c_void_p), H.shape[0], float(rho),
            rec.ctypes.data_as(c_void_p) if rec is not None else None, ctypes.byref(st))
        if rc < 0:
            raise DCGS2Error(rc, "dcgs2_arnoldi_steps")
        return rec, rc, st.as_dict()

    def qr_steps(self, B, j0: int, j1: int, Q, w, R, S, rho: float, record=True):
        """Steps j0..j1 of Alg. qr from the state (Q columns, w, S_{1:j0-2,j0-1}, rho);
        Q, w (device), R (numpy Fortran float64, >= j1-1 square) and S (numpy float64,
        >= j1-1 entries) are updated in place.  Returns (records or None, status, stats)."""
        m = B.shape[0]
        pb, ldb = _colmajor_args(B, "B")
        pq, ldq = _colmajor_args(Q, "Q")
        pw = _vec_ptr(w, "w", m)
        if (R.dtype != np.float64 or not R.flags.f_contiguous or R.shape[0] < j1 - 1
                or R.shape[1] < j1 - 1):
            raise ValueError("R must be a Fortran float64 array of >= (j1-1) x (j1-1)")
        if S.dtype != np.float64 or not S.flags.c_contiguous or S.size < j1 - 1:
            raise ValueError("S must be a contiguous float64 array of >= j1-1 entries")
        rec = np.empty((j1 - j0 + 1, 3 * j1 + 1)) if record else None
        st = Stats()
        rc = self._lib.dcgs2_qr_steps(
            self._h, m, j0, j1, pb, ldb, pq, ldq, pw, R.ctypes.data_as(c_void_p), R.shape[0],
            S.ctypes.data_as(c_void_p), float(rho),
            rec.ctypes.data_as(c_void_p) if rec is not None else None, ctypes.byref(st))
        if rc < 0:
            raise DCGS2Error(rc, "dcgs2_qr_steps")
        return rec, rc, st.as_dict()

    def gmres(self, op: Op, b, x, restart=50, rtol=1e-8, max_iters=100000):
        """Restarted GMRES(restart); x holds x0 on entry and the solution on return."""
        pb = _vec_ptr(b, "b", op.m)
        px = _vec_ptr(x, "x", op.m)
        info = GmresInfo()
        rc = self._lib.gmres_solve(self._h, ctypes.byref(op), pb, px, restart, rtol, max_iters,
                                   ctypes.byref(info))
        if rc < 0:
            raise DCGS2Error(rc, "gmres_solve")
        out = {k: getattr(info, k) for k, _ in GmresInfo._fields_ if k not in ("st", "pad")}
        out["stats"] = info.st.as_dict()
        return rc, out

    def krylov_schur(self, op: Op, v0, nev=10, ncv=60, keep=20, tol=1e-8, max_restarts=500):
        """Largest-magnitude eigenvalues; returns (eigs complex numpy, status, info)."""
        pv = _vec_ptr(v0, "v0", op.m)
        re = np.zeros(nev)
        im = np.zeros(nev)
        info = KsInfo()
        rc = self._lib.krylov_schur_eigs(self._h, ctypes.byref(op), nev, ncv, keep, tol,
                                         max_restarts, pv, re.ctypes.data_as(c_void_p),
                                         im.ctypes.data_as(c_void_p), ctypes.byref(info))
        if rc < 0:
            raise DCGS2Error(rc, "krylov_schur_eigs")
        out = {k: getattr(info, k) for k, _ in KsInfo._fields_ if k != "st"}
        out["stats"] = info.st.as_dict()
        return re + 1j * im, rc, out

    def gmres_batched(self, ops, restart, b, x, rtol=1e-8, max_iters=100000):
        """Batched GMRES over len(ops) stencil systems; b, x: device float64, concatenated
        (x holds x0 on entry, the solutions on return); restart: per instance.  Returns
        (status, list of per-instance info dicts)."""
        count = len(ops)
        arr = (Stencil2d * count)(*ops)
        rs = np.ascontiguousarray(restart, dtype=np.int32)
        total = int(sum(o.nx * o.ny for o in ops))
        pb = _vec_ptr(b, "b", total)
        px = _vec_ptr(x, "x", total)
        infos = (GmresInfo * count)()
        rc = self._lib.gmres_batched(self._h, count, arr, rs.ctypes.data_as(c_void_p), pb, px,
                                     rtol, max_iters, infos)
        if rc < 0:
            raise DCGS2Error(rc, "gmres_batched")
        out = []
        for inf in infos:
            d = {k: getattr(inf, k) for k, _ in GmresInfo._fields_ if k not in ("st", "pad")}
            d["stats"] = inf.st.as_dict()
            out.append(d)
        return rc, out

    def arnoldi_batched(self, ops, n, r0, Q=None):
        """Batched DCGS2 Arnoldi: ops (Stencil2d list), n (steps per instance), r0 (device,
        concatenated start vectors).  Q: device float64 buffer of
        batched_basis_size(ops, n) elements (allocated when None).  Returns
        (bases, H list, status, per-instance statuses, stats list); bases[b] is an
        m_b x (n_b+1) column-major view into Q."""
        import torch
        count = len(ops)
        arr = (Stencil2d * count)(*ops)
        nn = np.ascontiguousarray(n, dtype=np.int32)
        ms = [o.nx * o.ny for o in ops]
        pr = _vec_ptr(r0, "r0", int(sum(ms)))
        offs, total = batched_basis_offsets(ops, n)
        if Q is None:
            Q = torch.empty(total, dtype=torch.float64, device="cuda")
        if Q.dtype != torch.float64 or not Q.is_cuda or Q.numel() < total or not Q.is_contiguous():
            raise ValueError("Q must be a contiguous float64 device buffer of the batched size")
        hsz = [(int(k) + 1) * int(k) for k in nn]
        H = np.zeros(int(sum(hsz)))
        stat = np.zeros(count, dtype=np.int32)
        sts = (Stats * count)()
        rc = self._lib.dcgs2_arnoldi_batched(self._h, count, arr, nn.ctypes.data_as(c_void_p), pr,
                                             Q.data_ptr(), H.ctypes.data_as(c_void_p),
                                             stat.ctypes.data_as(c_void_p), sts)
        if rc < 0:
            raise DCGS2Error(rc, "dcgs2_arnoldi_batched")
        bases, Hs, h0 = [], [], 0
        for b, (m, k) in enumerate(zip(ms, nn)):
            ld = ((m + 63) // 64) * 64
            bases.append(Q[offs[b]:offs[b] + ld * (k + 1)].view(int(k) + 1, ld).t()[:m])
            Hs.append(H[h0:h0 + hsz[b]].reshape((int(k) + 1, int(k)), order="F"))
            h0 += hsz[b]
        return bases, Hs, rc, stat, [s.as_dict() for s in sts]

    def krylov_schur_batched(self, ops, v0, nev=10, ncv=60, keep=20, tol=1e-8,
                             max_restarts=500, use_graph=True):
        """Krylov-Schur on len(ops) stencil operators at once (Stencil2d descriptors).
        v0: CUDA float64 tensor, the start vectors concatenated in instance order.
        Returns (eigs complex numpy [count, nev], status, list of info dicts)."""
        count = len(ops)
        arr = (Stencil2d * count)(*ops)
        total = sum(o.nx * o.ny for o in ops)
        pv = _vec_ptr(v0, "v0", total)
        re = np.zeros((count, nev))
        im = np.zeros((count, nev))
        infos = (KsInfo * count)()
        rc = self._lib.krylov_schur_batched(self._h, count, arr, nev, ncv, keep, tol,
                                            max_restarts, pv, re.ctypes.data_as(c_void_p),
                                            im.ctypes.data_as(c_void_p), infos,
                                            1 if use_graph else 0)
        if rc < 0:
            raise DCGS2Error(rc, "krylov_schur_batched")
        out = []
        for inf in infos:
            d = {k: getattr(inf, k) for k, _ in KsInfo._fields_ if k != "st"}
            d["stats"] = inf.st.as_dict()
            out.append(d)
        return re + 1j * im, rc, out

    # ---- learned initial guess ------------------------------------------------------
    def guess_features(self, b, prm, n: int, nc: int, fdim: int):
        """b: CUDA float64 (count, n*n); prm: CUDA float32 (count, np).
        Returns (feat float32 (count, fdim), scale float64 (count,))."""
        import torch
        count = b.shape[0]
        np_ = prm.shape[1] if prm is not None else 0
        feat = torch.empty((count, fdim), dtype=torch.float32, device=b.device)
        scale = torch.empty(count, dtype=torch.float64, device=b.device)
        rc = self._lib.dcgs2_guess_features(self._h, count, n, nc, _ptr(b, torch.float64),
                                            _ptr(prm, torch.float32) if np_ else None, np_,
                                            fdim, feat.data_ptr(), scale.data_ptr())
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_guess_features")
        return feat, scale

    def guess_targets(self, x, scale, n: int, nc: int, gain: float = 1.0):
        import torch
        count = x.shape[0]
        t = torch.empty((count, nc * nc), dtype=torch.float32, device=x.device)
        rc = self._lib.dcgs2_guess_targets(self._h, count, n, nc, _ptr(x, torch.float64),
                                           _ptr(scale, torch.float64), gain, t.data_ptr())
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_guess_targets")
        return t

    def guess_prolong(self, y, scale, n: int, nc: int, gain: float = 1.0, out=None):
        import torch
        count = y.shape[0]
        x0 = out if out is not None else torch.empty((count, n * n), dtype=torch.float64,
                                                     device=y.device)
        rc = self._lib.dcgs2_guess_prolong(self._h, count, n, nc, _ptr(y, torch.float32),
                                           _ptr(scale, torch.float64), gain,
                                           _ptr(x0, torch.float64))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_guess_prolong")
        return x0

    def guess_guard(self, op: Op, b, x0, max_ratio=10.0):
        """Zero-guess fallback; returns (kept, ||b - A x0|| / ||b||)."""
        kept = c_int32()
        ratio = c_double()
        rc = self._lib.dcgs2_guess_guard(self._h, ctypes.byref(op), _vec_ptr(b, "b", op.m),
                                         _vec_ptr(x0, "x0", op.m), max_ratio,
                                         ctypes.byref(kept), ctypes.byref(ratio))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_guess_guard")
        return bool(kept.value), ratio.value

    def set_tuning(self, key: int, value: int):
        rc = self._lib.dcgs2_set_tuning(self._h, int(key), int(value))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_set_tuning")

    def get_tuning(self, key: int) -> int:
        v = c_int32()
        rc = self._lib.dcgs2_get_tuning(self._h, int(key), ctypes.byref(v))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_get_tuning")
        return v.value

    def set_basis_precision(self, bits: int):
        """Storage precision (32 or 64) of the internal bases of gmres / krylov_schur."""
        rc = self._lib.dcgs2_set_basis_precision(self._h, int(bits))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_set_basis_precision")

    def set_qr_schedule(self, one_pass: bool):
        rc = self._lib.dcgs2_set_qr_schedule(self._h, 1 if one_pass else 0)
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_set_qr_schedule")

    def profile(self, enable: bool = True):
        rc = self._lib.dcgs2_profile_enable(self._h, 1 if enable else 0)
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_profile_enable")

    def profile_read(self, reset: bool = True):
        """Per-kernel-class {launches, total_ms, bytes} accumulated since the last reset."""
        arr = (KernelStat * 16)()
        n = self._lib.dcgs2_profile_read(self._h, arr, 16, 1 if reset else 0)
        if n < 0:
            raise DCGS2Error(n, "dcgs2_profile_read")
        return {arr[i].name.decode(): dict(launches=arr[i].launches, total_ms=arr[i].total_ms,
                                          bytes=arr[i].bytes) for i in range(n)}

    def apply(self, op: Op, x, y):
        rc = self._lib.dcgs2_apply(self._h, ctypes.byref(op), _vec_ptr(x, "x", op.m),
                                   _vec_ptr(y, "y", op.m))
        if rc != OK:
            raise DCGS2Error(rc, "dcgs2_apply")
