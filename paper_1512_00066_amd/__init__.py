"""Python binding of libsrtc: semiring sparse tensor contraction on MI355X.

Argument marshalling only: every step of the computation runs in the HIP
library (``libsrtc.so``, C-ABI declared in ``include/srtc.h``).  PyTorch
provides device memory and the current stream; outputs the library
allocates come from torch through an allocator callback and are returned as
torch tensors.  Importing works without a GPU; calling needs one, and the
library must have been built (``paper_1512_00066_amd.build.build()``) --
there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsrtc.so")

# ------------------------------------------------------------------ enums --
PLUS_TIMES, MIN_PLUS, OR_AND, MAX_TIMES = 0, 1, 2, 3
SEMIRINGS = {"plus_times": PLUS_TIMES, "min_plus": MIN_PLUS, "or_and": OR_AND, "max_times": MAX_TIMES}
F64, F32, I32, BOOL8, BITS64, PATH64 = 0, 1, 2, 3, 4, 5
DENSE, COO_FMT, CSR_FMT = 0, 1, 2
NUM_SCHEDULES = 8
TRANSFORMS = {"recip": 0, "scale": 1, "add": 2, "fma": 3, "div_sum": 4}
NUM_FEATURES = 32

# int64 values are packed paths (weight << 32 | hops) for the (min,+) semiring
_TORCH_TO_DT = {torch.float64: F64, torch.float32: F32, torch.int32: I32, torch.uint8: BOOL8, torch.int64: PATH64}
_DT_TO_TORCH = {F64: torch.float64, F32: torch.float32, I32: torch.int32, BOOL8: torch.uint8, BITS64: torch.int64,
                PATH64: torch.int64}
_DT_CTYPE = {F64: ctypes.c_double, F32: ctypes.c_float, I32: ctypes.c_int32, BOOL8: ctypes.c_uint8,
             PATH64: ctypes.c_uint64}

STATUS = {0: "ok", -1: "invalid argument", -2: "invalid index string", -3: "dimension mismatch",
          -4: "value type not defined for the semiring", -5: "malformed sparse operand",
          -6: "output overlaps an input", -7: "out of memory", -8: "fixpoint not reached",
          -9: "unsupported", -10: "device error", -11: "request exceeds a fixed-size buffer"}


class SrtcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class NotConverged(SrtcError):
    def __init__(self, status, message, iters):
        super().__init__(status, message)
        self.iters = iters


class _Tensor(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("format", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("split", ctypes.c_int32), ("dims", ctypes.c_int64 * 8), ("nnz", ctypes.c_int64),
                ("coo_keys", ctypes.c_void_p), ("rowptr", ctypes.c_void_p), ("colidx", ctypes.c_void_p),
                ("vals", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("sorted", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("hub_tile", ctypes.c_int32)]


class _TrainCfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_PANEL = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(_Tensor),
                          ctypes.c_void_p)

_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1512_00066_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I32_, I64_ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        T = ctypes.POINTER(_Tensor)
        S = ctypes.c_char_p
        sig = {
            "srtc_ctx_create": ([ctypes.c_int, _ALLOC, _FREE, P, ctypes.POINTER(P)], ctypes.c_int),
            "srtc_ctx_destroy": ([P], ctypes.c_int),
            "srtc_last_error": ([P], ctypes.c_char_p),
            "srtc_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "srtc_fold": ([P, ctypes.c_int, P, S, T, S, S, T, P], ctypes.c_int),
            "srtc_contract": ([P, ctypes.c_int, P, ctypes.c_int, S, T, S, T, S, T, ctypes.POINTER(_Opts), P],
                              ctypes.c_int),
            "srtc_contract_noalloc": ([P, ctypes.c_int, P, ctypes.c_int, S, T, S, T, S, T, P], ctypes.c_int),
            "srtc_fixpoint": ([P, ctypes.c_int, P, T, T, I64_, I32_, ctypes.POINTER(I64_), P], ctypes.c_int),
            "srtc_fixpoint_ex": ([P, ctypes.c_int, P, T, T, I64_, I32_, I32_, ctypes.POINTER(I64_), P], ctypes.c_int),
            "srtc_contract_masked": ([P, ctypes.c_int, P, S, T, S, T, S, T, T, ctypes.POINTER(_Opts), P], ctypes.c_int),
            "srtc_bfs_levels": ([P, T, ctypes.POINTER(I64_), I32_, P, ctypes.POINTER(I32_), P], ctypes.c_int),
            "srtc_apsp_tiskin": ([P, P, T, P, P, ctypes.POINTER(I32_), ctypes.POINTER(I64_), P], ctypes.c_int),
            "srtc_transform": ([P, ctypes.c_int, ctypes.c_double, S, T, S, T, S, T, P], ctypes.c_int),
            "srtc_jacobi": ([P, T, T, T, ctypes.c_double, I64_, I32_, ctypes.POINTER(I64_),
                             ctypes.POINTER(ctypes.c_double), P], ctypes.c_int),
            "srtc_batch_contract": ([P, ctypes.c_int, P, I32_, T, T, T, S, S, S, ctypes.POINTER(I32_),
                                     ctypes.POINTER(_Opts), P], ctypes.c_int),
            "srtc_contract_panels": ([P, ctypes.c_int, P, S, T, S, T, S, ctypes.POINTER(_Opts), I64_, _PANEL, P, P],
                                     ctypes.c_int),
            "srtc_batch_fixpoint": ([P, ctypes.c_int, P, I32_, T, T, I64_, I32_, ctypes.POINTER(I64_), P],
                                    ctypes.c_int),
            "srtc_batch_autotune": ([P, ctypes.c_int, P, I32_, T, T, S, S, S, I32_, ctypes.POINTER(I32_),
                                     ctypes.POINTER(ctypes.c_float), P], ctypes.c_int),
            "srtc_features": ([P, ctypes.c_int, T, T, ctypes.POINTER(ctypes.c_float), P], ctypes.c_int),
            "srtc_autotune": ([P, ctypes.c_int, P, T, T, I32_, ctypes.POINTER(I32_), ctypes.POINTER(ctypes.c_float),
                               P], ctypes.c_int),
            "srtc_select": ([P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(I32_)], ctypes.c_int),
            "srtc_selector_train": ([P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), I32_,
                                     ctypes.POINTER(_TrainCfg), ctypes.POINTER(ctypes.c_float), P], ctypes.c_int),
            "srtc_selector_save": ([P, S], ctypes.c_int),
            "srtc_selector_load": ([P, S], ctypes.c_int),
            "srtc_mlp_forward": ([P, P, P, I32_, P, P], ctypes.c_int),
            "srtc_mlp_loss_grad": ([P, P, P, P, I32_, P, P, P], ctypes.c_int),
            "srtc_mlp_adam_step": ([P, P, P, P, P, I64_, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, P], ctypes.c_int),
            "srtc_profile_enable": ([P, I32_], ctypes.c_int),
            "srtc_profile_query": ([P, I32_, ctypes.c_char_p, I32_, ctypes.POINTER(I64_),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "srtc_mlp_num_params": ([], I64_),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


# ------------------------------------------------------------- tensors --
@dataclass
class CSR:
    """A CSR tensor on the device: rows = leading ``split`` modes."""
    rowptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor
    dims: tuple
    split: int = 1
    _keep: list = field(default_factory=list, repr=False)

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @property
    def shape(self):
        r = int(np.prod(self.dims[: self.split], dtype=np.int64))
        c = int(np.prod(self.dims[self.split:], dtype=np.int64))
        return (r, c)

    def to_host(self):
        return (self.rowptr.cpu().numpy(), self.col.cpu().numpy(), self.val.cpu().numpy())


@dataclass
class COO:
    """Index-value pairs: linearized keys (last mode fastest) and values."""
    keys: torch.Tensor
    val: torch.Tensor
    dims: tuple


def csr_from_host(rowptr, col, val, dims, device="cuda", split=1) -> CSR:
    return CSR(torch.as_tensor(np.ascontiguousarray(rowptr, dtype=np.int64), device=device),
               torch.as_tensor(np.ascontiguousarray(col, dtype=np.int32), device=device),
               torch.as_tensor(np.ascontiguousarray(val), device=device), tuple(int(d) for d in dims), split)


def _dt(t: torch.Tensor) -> int:
    try:
        return _TORCH_TO_DT[t.dtype]
    except KeyError:
        raise SrtcError(-4, f"unsupported value type {t.dtype}")


def _ptr(t: Optional[torch.Tensor]):
    if t is None or t.numel() == 0:
        return None
    if not t.is_contiguous():
        raise SrtcError(-1, "tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _desc(x) -> _Tensor:
    d = _Tensor()
    if isinstance(x, CSR):
        d.order = len(x.dims)
        d.format = CSR_FMT
        d.dtype = _dt(x.val)
        d.split = x.split
        for i, v in enumerate(x.dims):
            d.dims[i] = int(v)
        d.nnz = x.nnz
        d.rowptr = _ptr(x.rowptr)
        d.colidx = _ptr(x.col)
        d.vals = _ptr(x.val)
    elif isinstance(x, COO):
        d.order = len(x.dims)
        d.format = COO_FMT
        d.dtype = _dt(x.val)
        for i, v in enumerate(x.dims):
            d.dims[i] = int(v)
        d.nnz = int(x.keys.numel())
        d.coo_keys = _ptr(x.keys)
        d.vals = _ptr(x.val)
    elif isinstance(x, torch.Tensor):
        d.order = x.dim()
        d.format = DENSE
        d.dtype = _dt(x)
        for i, v in enumerate(x.shape):
            d.dims[i] = int(v)
        d.vals = _ptr(x)
    else:
        raise SrtcError(-1, f"not a tensor: {type(x)}")
    return d


def _add_id(add_id, dtype):
    if add_id is None:
        return None
    return ctypes.byref(_DT_CTYPE[dtype](add_id))


def pack_path(weight, hops):
    """Packed (min,+) path values (int64): weight << 32 | hops."""
    w = torch.as_tensor(weight).to(torch.int64)
    h = torch.as_tensor(hops).to(torch.int64)
    return (w << 32) | h


def unpack_path(p: torch.Tensor):
    """(weight, hops) of packed path values."""
    return (p >> 32).to(torch.int32), (p & 0xFFFFFFFF).to(torch.int32)


def _sr(semiring) -> int:
    if isinstance(semiring, str):
        return SEMIRINGS[semiring]
    return int(semiring)


class Context:
    """A library context on one device; device buffers it returns are torch
    tensors allocated on that device."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        self._live = {}
        live = self._live
        dev = self.device
        # number of allocator callbacks so far (tests check calls that must
        # allocate nothing)
        self._nalloc = nalloc = [0]

        def _a(user, nbytes):
            t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=dev)
            p = t.data_ptr()
            live[p] = t
            nalloc[0] += 1
            return p

        def _f(user, ptr):
            live.pop(ptr, None)

        self._cb = (_ALLOC(_a), _FREE(_f))
        h = ctypes.c_void_p()
        st = lib().srtc_ctx_create(device, self._cb[0], self._cb[1], None, ctypes.byref(h))
        if st != 0:
            raise SrtcError(st, "context creation failed")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.srtc_ctx_destroy(h)
            self._h = None

    @property
    def allocations(self) -> int:
        """Device allocations the library has requested from this context."""
        return self._nalloc[0]

    # -------------------------------------------------------- internals --
    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _check(self, st, extra=None):
        if st != 0:
            msg = lib().srtc_last_error(self._h).decode()
            if st == -8:
                raise NotConverged(st, msg, extra)
            raise SrtcError(st, msg)

    def _take(self, ptr, count, dtype, base=None, offset_bytes=0):
        """Torch tensor over library output memory (owned via the callback)."""
        if base is None:
            t = self._live.pop(ptr)
            offset_bytes = 0
        else:
            t = base
        esize = torch.empty((), dtype=dtype).element_size()
        if count == 0:
            return torch.empty(0, dtype=dtype, device=self.device)
        return t[offset_bytes: offset_bytes + count * esize].view(dtype)

    def _csr_out(self, d: _Tensor) -> CSR:
        order = d.order
        dims = tuple(int(d.dims[i]) for i in range(order))
        rows = int(np.prod(dims[: d.split], dtype=np.int64))
        rp = self._take(d.rowptr, rows + 1, torch.int64)
        col = self._take(d.colidx, d.nnz, torch.int32) if d.nnz else self._drop(d.colidx, torch.int32)
        val = self._take(d.vals, d.nnz, _DT_TO_TORCH[d.dtype]) if d.nnz else self._drop(d.vals, _DT_TO_TORCH[d.dtype])
        return CSR(rp, col, val, dims, d.split)

    def _drop(self, ptr, dtype):
        if ptr:
            self._live.pop(ptr, None)
        return torch.empty(0, dtype=dtype, device=self.device)

    # --------------------------------------------------------------- API --
    def fold(self, semiring, src, isrc: str, rows: str, cols: str, add_id=None) -> CSR:
        """Fold a COO/CSR tensor into a CSR matrix (rows/cols name its modes)."""
        sd = _desc(src)
        out = _Tensor()
        st = lib().srtc_fold(self._h, _sr(semiring), _add_id(add_id, sd.dtype), isrc.encode(), ctypes.byref(sd),
                             rows.encode(), cols.encode(), ctypes.byref(out), self._stream())
        self._check(st)
        return self._csr_out(out)

    def contract(self, semiring, ia: str, A, ib: str, B, ic: str, C=None, accumulate=False, add_id=None,
                 schedule: int = -1, sorted: bool = True, out_dims=None, validate: bool = False,
                 hub_tile: int = 0):
        """C[ic] (+)= A[ia] (x) B[ib].  Sparse x sparse returns a CSR; with a
        dense operand C must be a preallocated dense tensor (returned).
        validate: check the sparse operands' structure first.  hub_tile: the
        size of the dense hub block formed on the matrix cores ((+,x) sparse
        products; 0 = none)."""
        ad, bd = _desc(A), _desc(B)
        opts = _Opts(schedule, 1 if sorted else 0, 1 if validate else 0, int(hub_tile))
        if C is None:
            # sparse result: dims of C from the index strings
            ext = {}
            for s_, t in ((ia, A), (ib, B)):
                dims = t.dims if not isinstance(t, torch.Tensor) else tuple(t.shape)
                for ch, e in zip(s_, dims):
                    ext[ch] = int(e)
            cd = _Tensor()
            cd.order = len(ic)
            cd.format = CSR_FMT
            cd.dtype = ad.dtype
            for i, ch in enumerate(ic):
                cd.dims[i] = ext.get(ch, 1)
        else:
            cd = _desc(C)
        st = lib().srtc_contract(self._h, _sr(semiring), _add_id(add_id, ad.dtype), int(bool(accumulate)),
                                 ia.encode(), ctypes.byref(ad), ib.encode(), ctypes.byref(bd), ic.encode(),
                                 ctypes.byref(cd), ctypes.byref(opts), self._stream())
        self._check(st)
        if C is None or isinstance(C, CSR):
            return self._csr_out(cd)
        return C

    def contract_noalloc(self, semiring, ia: str, A, ib: str, B, ic: str, C, accumulate=False, add_id=None):
        """C[ic] (+)= A[ia] (x) B[ib] for CSR A and dense B and C, with no
        device allocation (the library's fixed per-device buffer holds the
        plan).  Layouts: ia = C's row letters then the inner ones, ib = the
        inner letters then C's column letters, ic = rows then columns.
        Returns C."""
        ad, bd, cd = _desc(A), _desc(B), _desc(C)
        st = lib().srtc_contract_noalloc(self._h, _sr(semiring), _add_id(add_id, ad.dtype), int(bool(accumulate)),
                                         ia.encode(), ctypes.byref(ad), ib.encode(), ctypes.byref(bd), ic.encode(),
                                         ctypes.byref(cd), self._stream())
        self._check(st)
        return C

    def contract_panels(self, semiring, ia: str, A, ib: str, B, ic: str, consume, panel_products: int = 0,
                        add_id=None, schedule: int = -1, sorted: bool = True, validate: bool = False) -> int:
        """C[ic] = A[ia] (x) B[ib] streamed by row panels: ``consume(row0, P)``
        receives each panel P (a CSR of C's rows row0 .. row0 + P.shape[0] - 1,
        folded to a matrix) and may keep it; returning False stops the
        product (SrtcError).  Panels hold at most ``panel_products`` products
        each (0: 2^31).  Returns the number of panels."""
        ad, bd = _desc(A), _desc(B)
        opts = _Opts(schedule, 1 if sorted else 0, 1 if validate else 0, 0)
        errors = []
        count = [0]

        def _cb(user, row0, nrows, desc, stream):
            try:
                P = self._csr_out(desc.contents)
                count[0] += 1
                return 1 if consume(int(row0), P) is False else 0
            except BaseException as e:  # noqa: BLE001 -- re-raised after the call
                errors.append(e)
                return 1

        cb = _PANEL(_cb)
        st = lib().srtc_contract_panels(self._h, _sr(semiring), _add_id(add_id, ad.dtype), ia.encode(),
                                        ctypes.byref(ad), ib.encode(), ctypes.byref(bd), ic.encode(),
                                        ctypes.byref(opts), int(panel_products), cb, None, self._stream())
        if errors:
            raise errors[0]
        self._check(st)
        return count[0]

    def contract_masked(self, semiring, ia: str, A, ib: str, B, ic: str, M, add_id=None,
                        validate: bool = False) -> "CSR":
        """C[ic] = M (.) (A[ia] (x) B[ib]): only positions in M's pattern
        (M sparse, indexed like C; its values are ignored)."""
        ad, bd, md = _desc(A), _desc(B), _desc(M)
        opts = _Opts(-1, 1, 1 if validate else 0, 0)
        cd = _Tensor()
        cd.order = len(ic)
        cd.format = CSR_FMT
        cd.dtype = ad.dtype
        mdims = M.dims if not isinstance(M, torch.Tensor) else tuple(M.shape)
        for i in range(len(ic)):
            cd.dims[i] = int(mdims[i])
        st = lib().srtc_contract_masked(self._h, _sr(semiring), _add_id(add_id, ad.dtype), ia.encode(),
                                        ctypes.byref(ad), ib.encode(), ctypes.byref(bd), ic.encode(),
                                        ctypes.byref(md), ctypes.byref(cd), ctypes.byref(opts), self._stream())
        self._check(st)
        return self._csr_out(cd)

    def fixpoint(self, semiring, A: CSR, X: torch.Tensor, max_iters: int = 0, steps_per_check: int = 4,
                 add_id=None, changed_rows_only: bool = False) -> int:
        """X <- X (+) A (x) X until unchanged (in place); returns the step count.
        changed_rows_only: each step gathers only from rows that changed in
        the previous one (same iterates and result)."""
        ad, xd = _desc(A), _desc(X)
        it = ctypes.c_int64(0)
        st = lib().srtc_fixpoint_ex(self._h, _sr(semiring), _add_id(add_id, ad.dtype), ctypes.byref(ad),
                                    ctypes.byref(xd), int(max_iters), int(steps_per_check),
                                    1 if changed_rows_only else 0, ctypes.byref(it), self._stream())
        self._check(st, it.value)
        return it.value

    def bfs_levels(self, A: CSR, sources: Sequence[int]):
        """Levels (n x nsrc int32, -1 unreachable) and depth of a multi-source BFS."""
        src = np.ascontiguousarray(sources, dtype=np.int64)
        n = A.shape[0]
        levels = torch.empty((n, src.size), dtype=torch.int32, device=self.device)
        depth = ctypes.c_int32(0)
        ad = _desc(A)
        st = lib().srtc_bfs_levels(self._h, ctypes.byref(ad), src.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   int(src.size), _ptr(levels), ctypes.byref(depth), self._stream())
        self._check(st)
        return levels, depth.value

    def transform(self, op: str, C, A=None, ia: str = "", B=None, ib: str = "", ic: Optional[str] = None,
                  alpha: float = 1.0):
        """Elementwise transform of C in place (op: recip, scale, add, fma,
        div_sum; see srtc_transform); A and B broadcast over C's letters."""
        cd = _desc(C)
        ad = _desc(A) if A is not None else None
        bd = _desc(B) if B is not None else None
        if ic is None:
            ic = "abcdefgh"[:cd.order]
        st = lib().srtc_transform(self._h, TRANSFORMS[op], float(alpha), ia.encode(),
                                  ctypes.byref(ad) if ad is not None else None, ib.encode(),
                                  ctypes.byref(bd) if bd is not None else None, ic.encode(), ctypes.byref(cd),
                                  self._stream())
        self._check(st)
        return C

    def jacobi(self, A, b: torch.Tensor, x: torch.Tensor, tol: float = 1e-6, max_iters: int = 0,
               steps_per_check: int = 8):
        """Jacobi iteration for A x = b from x (updated in place); returns
        (updates, residual norm)."""
        ad, bd, xd = _desc(A), _desc(b), _desc(x)
        it = ctypes.c_int64(0)
        rr = ctypes.c_double(0.0)
        st = lib().srtc_jacobi(self._h, ctypes.byref(ad), ctypes.byref(bd), ctypes.byref(xd), float(tol),
                               int(max_iters), int(steps_per_check), ctypes.byref(it), ctypes.byref(rr),
                               self._stream())
        self._check(st, it.value)
        return it.value, rr.value

    def apsp_tiskin(self, A, add_id=None, hops: bool = True, round_nnz: Optional[list] = None):
        """All-pairs lightest paths by path doubling: (D, H or None, rounds).
        A: n x n int32 COO or CSR, entry (i, j) = weight of edge j -> i;
        D[i, j] = weight of the lightest path j -> i (add_id, default
        INT32_MAX // 2, where none), H[i, j] = its hop count (-1 where none).
        round_nnz (a list, optional) receives the sparse factor's entries per
        product."""
        ad = _desc(A)
        n = int(A.dims[0])
        D = torch.empty((n, n), dtype=torch.int32, device=self.device)
        H = torch.empty((n, n), dtype=torch.int32, device=self.device) if hops else None
        r = ctypes.c_int32(0)
        rn = (ctypes.c_int64 * 64)()
        st = lib().srtc_apsp_tiskin(self._h, _add_id(add_id, I32), ctypes.byref(ad), _ptr(D), _ptr(H),
                                    ctypes.byref(r), rn, self._stream())
        self._check(st)
        if round_nnz is not None:
            round_nnz[:] = [int(x) for x in rn[:r.value]]
        return D, H, r.value

    def batch_contract(self, semiring, As: List[CSR], Bs: List[CSR], add_id=None, schedule: int = -1,
                       sorted: bool = True, ia: str = "ik", ib: str = "kj", ic: str = "ij",
                       schedules: Optional[Sequence[int]] = None, validate: bool = False) -> List[CSR]:
        """C_b[ic] = A_b[ia] (x) B_b[ib] for every instance in one set of
        launches; ``schedules`` (one id per instance, -1 = choose) or one
        ``schedule`` for all."""
        n = len(As)
        arrA = (_Tensor * n)(*[_desc(a) for a in As])
        arrB = (_Tensor * n)(*[_desc(b) for b in Bs])
        arrC = (_Tensor * n)()
        opts = _Opts(schedule, 1 if sorted else 0, 1 if validate else 0, 0)
        sch = None
        if schedules is not None:
            if len(schedules) != n:
                raise SrtcError(-1, "one schedule per instance")
            sch = (ctypes.c_int32 * n)(*[int(x) for x in schedules])
        st = lib().srtc_batch_contract(self._h, _sr(semiring), _add_id(add_id, arrA[0].dtype), n, arrA, arrB, arrC,
                                       ia.encode(), ib.encode(), ic.encode(), sch, ctypes.byref(opts),
                                       self._stream())
        self._check(st)
        c0 = arrC[0]
        base_rp = self._live.pop(c0.rowptr)
        base_col = self._live.pop(c0.colidx)
        base_val = self._live.pop(c0.vals)
        dt = _DT_TO_TORCH[c0.dtype]
        es = torch.empty((), dtype=dt).element_size()
        out = []
        for b in range(n):
            d = arrC[b]
            rows = int(d.dims[0])
            rp = self._take(None, rows + 1, torch.int64, base_rp, d.rowptr - c0.rowptr)
            col = self._take(None, d.nnz, torch.int32, base_col, d.colidx - c0.colidx)
            val = self._take(None, d.nnz, dt, base_val, d.vals - c0.vals)
            out.append(CSR(rp, col, val, (int(d.dims[0]), int(d.dims[1])), 1, [base_rp, base_col, base_val]))
        return out

    def batch_fixpoint(self, semiring, As: List[CSR], Xs: List[torch.Tensor], max_iters: int = 0,
                       steps_per_check: int = 4, add_id=None) -> List[int]:
        n = len(As)
        arrA = (_Tensor * n)(*[_desc(a) for a in As])
        arrX = (_Tensor * n)(*[_desc(x) for x in Xs])
        iters = (ctypes.c_int64 * n)()
        st = lib().srtc_batch_fixpoint(self._h, _sr(semiring), _add_id(add_id, arrA[0].dtype), n, arrA, arrX,
                                       int(max_iters), int(steps_per_check), iters, self._stream())
        self._check(st, list(iters))
        return list(iters)

    def features(self, semiring, A: CSR, B: CSR) -> np.ndarray:
        out = (ctypes.c_float * NUM_FEATURES)()
        ad, bd = _desc(A), _desc(B)
        st = lib().srtc_features(self._h, _sr(semiring), ctypes.byref(ad), ctypes.byref(bd), out, self._stream())
        self._check(st)
        return np.array(out[:], dtype=np.float32)

    def autotune(self, semiring, A: CSR, B: CSR, reps: int = 10, add_id=None):
        """(best schedule, median ms per schedule)."""
        ad, bd = _desc(A), _desc(B)
        best = ctypes.c_int32(-1)
        times = (ctypes.c_float * NUM_SCHEDULES)()
        st = lib().srtc_autotune(self._h, _sr(semiring), _add_id(add_id, ad.dtype), ctypes.byref(ad),
                                 ctypes.byref(bd), int(reps), ctypes.byref(best), times, self._stream())
        self._check(st)
        return best.value, np.array(times[:], dtype=np.float32)

    def batch_autotune(self, semiring, As: List[CSR], Bs: List[CSR], reps: int = 3, add_id=None,
                       ia: str = "ik", ib: str = "kj", ic: str = "ij"):
        """(best schedule, median ms per schedule) for the whole batch as
        batch_contract forms it with one schedule; the winner is cached, so a
        later batch_contract of the batch without schedules takes it."""
        n = len(As)
        arrA = (_Tensor * n)(*[_desc(a) for a in As])
        arrB = (_Tensor * n)(*[_desc(b) for b in Bs])
        best = ctypes.c_int32(-1)
        times = (ctypes.c_float * NUM_SCHEDULES)()
        st = lib().srtc_batch_autotune(self._h, _sr(semiring), _add_id(add_id, arrA[0].dtype), n, arrA, arrB,
                                       ia.encode(), ib.encode(), ic.encode(), int(reps), ctypes.byref(best), times,
                                       self._stream())
        self._check(st)
        return best.value, np.array(times[:], dtype=np.float32)

    def select(self, features) -> int:
        f = np.ascontiguousarray(features, dtype=np.float32)
        out = ctypes.c_int32(-1)
        st = lib().srtc_select(self._h, f.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(out))
        self._check(st)
        return out.value

    def selector_train(self, X, T, epochs=200, batch=128, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                       seed=0) -> float:
        X = np.ascontiguousarray(X, dtype=np.float32)
        T = np.ascontiguousarray(T, dtype=np.float32)
        cfg = _TrainCfg(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps), int(seed))
        loss = ctypes.c_float(0)
        st = lib().srtc_selector_train(self._h, X.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                       T.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(X.shape[0]),
                                       ctypes.byref(cfg), ctypes.byref(loss), self._stream())
        self._check(st)
        return loss.value

    def selector_save(self, path: str):
        self._check(lib().srtc_selector_save(self._h, path.encode()))

    def selector_load(self, path: str):
        self._check(lib().srtc_selector_load(self._h, path.encode()))

    def mlp_forward(self, params: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
        Y = torch.empty((X.shape[0], NUM_SCHEDULES), dtype=torch.float32, device=self.device)
        self._check(lib().srtc_mlp_forward(self._h, _ptr(params), _ptr(X), int(X.shape[0]), _ptr(Y),
                                           self._stream()))
        return Y

    def mlp_adam_step(self, params: torch.Tensor, grads: torch.Tensor, m1: torch.Tensor, m2: torch.Tensor,
                      step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        """One Adam update of params, m1 and m2 in place (step >= 1)."""
        self._check(lib().srtc_mlp_adam_step(self._h, _ptr(params), _ptr(grads), _ptr(m1), _ptr(m2), int(step),
                                             float(lr), float(beta1), float(beta2), float(eps), self._stream()))

    def mlp_loss_grad(self, params: torch.Tensor, X: torch.Tensor, T: torch.Tensor):
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        grads = torch.empty_like(params)
        self._check(lib().srtc_mlp_loss_grad(self._h, _ptr(params), _ptr(X), _ptr(T), int(X.shape[0]),
                                             _ptr(loss), _ptr(grads), self._stream()))
        return loss, grads


def mlp_num_params() -> int:
    return int(lib().srtc_mlp_num_params())


_default = None


def context() -> Context:
    """A process-wide context on cuda:0."""
    global _default
    if _default is None:
        _default = Context(0)
    return _default
