"""ctypes binding of libspc5hip.so. Argument marshalling only: every step of
conversion, planning and the products runs in the library's HIP kernels;
torch tensors only carry device memory, and torch's current stream is the
stream the library enqueues on.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_int32, c_int64, c_void_p

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libspc5hip.so")
SHAPES = ((1, 8), (2, 4), (2, 8), (4, 4), (4, 8), (8, 4))
F32, F64 = 0, 1


class SpcError(RuntimeError):
    def __init__(self, code: int, name: str, detail: str):
        super().__init__(f"{name} ({code}): {detail}")
        self.code = code
        self.name = name


class BetaView(ctypes.Structure):
    _fields_ = [("r", c_int32), ("c", c_int32), ("dtype", c_int32), ("reserved", c_int32),
                ("n_rows", c_int64), ("n_cols", c_int64), ("nnz", c_int64), ("n_blocks", c_int64),
                ("block_rowptr", c_void_p), ("block_colidx", c_void_p),
                ("block_masks", c_void_p), ("values", c_void_p)]


class PlanParams(ctypes.Structure):
    _fields_ = [("tile_bits", c_int32), ("tile_order", c_int32), ("mode", c_int32),
                ("wave_chunks", c_int32), ("pipeline", c_int32), ("cu_groups", c_int32),
                ("wave_tiles", c_int32), ("spmm_path", c_int32)]


class TuneRecord(ctypes.Structure):
    _fields_ = [("params", PlanParams), ("us", ctypes.c_float), ("n_tiles", c_int32)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "spc_status_string": (c_char_p, [c_int32]),
    "spc_last_error": (c_char_p, []),
    "spc_version": (c_int32, []),
    "spc_shape_index": (c_int32, [c_int32, c_int32]),
    "spc_mask_bytes": (c_int64, [c_int32, c_int32, c_int64]),
    "spc_beta_count": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_void_p, c_void_p, c_void_p,
                                 POINTER(c_int64), c_void_p]),
    "spc_csr_to_beta": (c_int32, [c_int32, c_int32, c_int32, c_int64, c_int64, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "spc_beta_to_csr": (c_int32, [POINTER(BetaView), c_void_p, c_void_p, c_void_p, c_void_p]),
    "spc_rcm_order": (c_int32, [c_int64, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "spc_csr_permute": (c_int32, [c_int64, c_int64, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p]),
    "spc_permute_vector": (c_int32, [c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "spc_plan_create": (c_int32, [POINTER(BetaView), POINTER(PlanParams), POINTER(c_void_p), c_void_p]),
    "spc_plan_destroy": (c_int32, [c_void_p]),
    "spc_plan_default_params": (c_int32, [POINTER(BetaView), POINTER(PlanParams)]),
    "spc_plan_info": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int32)]),
    "spc_spmv_beta": (c_int32, [POINTER(BetaView), c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "spc_spmm_beta": (c_int32, [POINTER(BetaView), c_void_p, c_int32, c_void_p, c_int64, c_void_p, c_int64,
                                c_int32, c_void_p]),
    "spc_cg_workspace_bytes": (c_int64, [c_int64, c_int32, c_int32]),
    "spc_cg_solve": (c_int32, [POINTER(BetaView), c_void_p, c_int32, c_void_p, c_int64, c_void_p, c_int64,
                               ctypes.c_double, c_int32, c_int32, c_int32, c_void_p, c_int64,
                               POINTER(c_int32), POINTER(ctypes.c_double), POINTER(c_int32), c_void_p]),
    "spc_time_spmv": (c_int32, [POINTER(BetaView), c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                POINTER(ctypes.c_float), c_void_p]),
    "spc_autotune": (c_int32, [POINTER(BetaView), c_void_p, c_void_p, c_int32, POINTER(PlanParams),
                               POINTER(ctypes.c_float), c_void_p, c_int32, POINTER(c_int32), c_void_p]),
    "spc_matrix_features": (c_int32, [c_int64, c_int64, c_int64, c_void_p, c_void_p, POINTER(ctypes.c_float),
                                      POINTER(c_int64), c_void_p]),
    "spc_matrix_features_noalloc": (c_int32, [c_int64, c_int64, c_int64, c_void_p, c_void_p,
                                              POINTER(ctypes.c_float), POINTER(c_int64), c_void_p]),
    "spc_matrix_features_noalloc_max_rows": (c_int64, []),
    "spc_batch_create": (c_int32, [c_int32, POINTER(BetaView), POINTER(PlanParams), c_int32, POINTER(c_void_p),
                                   c_void_p]),
    "spc_batch_destroy": (c_int32, [c_void_p]),
    "spc_batch_info": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int32), POINTER(c_int32)]),
    "spc_batch_set_kernel": (c_int32, [c_void_p, c_int32]),
    "spc_batch_set_vectors": (c_int32, [c_void_p, POINTER(c_void_p), POINTER(c_void_p)]),
    "spc_spmv_batched": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p]),
    "spc_mlp_standardizer": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "spc_mlp_targets": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "spc_mlp_loss_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                    POINTER(c_int32), c_int32, c_void_p, c_void_p, c_void_p]),
    "spc_mlp_train": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, ctypes.c_float, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_int32, c_int32, POINTER(c_int32), c_int32, c_int32, c_void_p, c_void_p]),
    "spc_mlp_infer": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p,
                                c_void_p]),
    "spc_class_shape": (c_int32, [c_int32]),
    "spc_class_mode": (c_int32, [c_int32]),
    "spc_selector_create": (c_int32, [POINTER(c_void_p)]),
    "spc_selector_destroy": (c_int32, [c_void_p]),
    "spc_selector_fit_interp": (c_int32, [c_void_p, c_int32, c_int32, POINTER(ctypes.c_double),
                                          POINTER(ctypes.c_double), c_int32]),
    "spc_selector_interp_coeffs": (c_int32, [c_void_p, POINTER(ctypes.c_double), POINTER(ctypes.c_double),
                                             POINTER(ctypes.c_double), POINTER(c_int32)]),
    "spc_selector_n_classes": (c_int32, [c_void_p, c_int32]),
    "spc_selector_set_mlp": (c_int32, [c_void_p, c_int32, POINTER(ctypes.c_float), POINTER(ctypes.c_float),
                                       POINTER(ctypes.c_float)]),
    "spc_select_kernel": (c_int32, [c_void_p, POINTER(ctypes.c_float), c_int32, POINTER(c_int32),
                                    POINTER(ctypes.c_float), c_void_p]),
    "spc_stream_create_cu": (c_int32, [c_int32, POINTER(c_void_p)]),
    "spc_stream_destroy": (c_int32, [c_void_p]),
    "spc_device_cu_count": (c_int32, []),
    "spc_selector_fit_interp2d": (c_int32, [c_void_p, c_int32, POINTER(ctypes.c_double), POINTER(ctypes.c_double),
                                            POINTER(ctypes.c_double), c_int32, c_int32]),
    "spc_selector_interp2d_coeffs": (c_int32, [c_void_p, POINTER(ctypes.c_double), POINTER(ctypes.c_double),
                                               POINTER(ctypes.c_double), POINTER(ctypes.c_double)]),
    "spc_select_kernel_at": (c_int32, [c_void_p, POINTER(ctypes.c_float), ctypes.c_double, POINTER(c_int32),
                                       POINTER(ctypes.c_float)]),
}


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1801_01134_amd.build` (there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def register(name: str, restype, argtypes):
    """Declare the signature of a further entry point (used by sibling modules)."""
    _SIGS[name] = (restype, argtypes)
    if _lib is not None:
        f = getattr(_lib, name)
        f.restype = restype
        f.argtypes = argtypes


def check(status: int):
    if status != 0:
        L = lib()
        raise SpcError(status, L.spc_status_string(status).decode(), L.spc_last_error().decode())


def stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _dtype_code(dt) -> int:
    if dt == torch.float64:
        return F64
    if dt == torch.float32:
        return F32
    raise TypeError(f"unsupported value dtype {dt}")


def _dev(a, dtype=None, device="cuda"):
    if isinstance(a, torch.Tensor):
        t = a.to(device=device)
        if dtype is not None:
            t = t.to(dtype)
        return t.contiguous()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device).contiguous()


def mask_bytes(r: int, c: int, n_blocks: int) -> int:
    return int(lib().spc_mask_bytes(r, c, n_blocks))


class Plan:
    """A tile plan (library-owned) for one BetaMatrix."""

    def __init__(self, A: "BetaMatrix", tile_bits: int = 0, tile_order: int = 0, mode: int = 0,
                 wave_chunks: int = 0, pipeline: int = 0, cu_groups: int = 0, wave_tiles: int = 0,
                 spmm_path: int = 0):
        self._A = A
        self._view = A.view()
        p = PlanParams(tile_bits, tile_order, mode, wave_chunks, pipeline, cu_groups, wave_tiles, spmm_path)
        h = c_void_p()
        check(lib().spc_plan_create(ctypes.byref(self._view), ctypes.byref(p), ctypes.byref(h),
                                    stream_ptr()))
        self.handle = h

    def info(self) -> dict:
        nt, nl, tb = c_int64(), c_int64(), c_int32()
        check(lib().spc_plan_info(self.handle, ctypes.byref(nt), ctypes.byref(nl), ctypes.byref(tb)))
        return {"n_tiles": nt.value, "n_long": nl.value, "tile_bits": tb.value}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.spc_plan_destroy(h)
            self.handle = None


class BetaMatrix:
    """A beta(r,c) matrix in device tensors (the arrays of the storage format)."""

    def __init__(self, r, c, n_rows, n_cols, block_rowptr, block_colidx, block_masks, values):
        self.r, self.c = int(r), int(c)
        self.n_rows, self.n_cols = int(n_rows), int(n_cols)
        self.block_rowptr = block_rowptr
        self.block_colidx = block_colidx
        self.block_masks = block_masks
        self.values = values
        self._plans = {}

    @property
    def dtype(self):
        return self.values.dtype

    @property
    def nnz(self) -> int:
        return int(self.values.numel())

    @property
    def n_blocks(self) -> int:
        return int(self.block_colidx.numel())

    @property
    def shape_index(self) -> int:
        return SHAPES.index((self.r, self.c))

    def view(self) -> BetaView:
        # the masks array always exists (it carries the read-ahead padding);
        # the other arrays may be empty, and then have no address
        return BetaView(self.r, self.c, _dtype_code(self.values.dtype), 0, self.n_rows, self.n_cols,
                        self.nnz, self.n_blocks, self.block_rowptr.data_ptr(),
                        self.block_colidx.data_ptr() if self.n_blocks else None,
                        self.block_masks.data_ptr(),
                        self.values.data_ptr() if self.nnz else None)

    def plan(self, tile_bits: int = 0, tile_order: int = 0, mode: int = 0, wave_chunks: int = 0,
             pipeline: int = 0, cu_groups: int = 0, wave_tiles: int = 0, spmm_path: int = 0) -> Plan:
        key = (tile_bits, tile_order, mode, wave_chunks, pipeline, cu_groups, wave_tiles, spmm_path)
        if key not in self._plans:
            self._plans[key] = Plan(self, tile_bits, tile_order, mode, wave_chunks, pipeline, cu_groups, wave_tiles,
                                    spmm_path)
        return self._plans[key]

    def default_params(self) -> dict:
        """The library's default plan parameters for this matrix (from its sizes)."""
        v = self.view()
        p = PlanParams()
        check(lib().spc_plan_default_params(ctypes.byref(v), ctypes.byref(p)))
        return _params_dict(p)

    def default_plan(self) -> Plan:
        return plan_from(self, self.default_params())

    def nbytes(self) -> int:
        """Bytes of the four arrays as Eq. (1) counts them (masks unpadded)."""
        return (self.values.numel() * self.values.element_size() + self.block_rowptr.numel() * 4
                + self.block_colidx.numel() * 4 + self.n_blocks * self.r * self.c // 8)


def csr_to_beta(r: int, c: int, rowptr, colidx, values, n_cols: int, dtype=None,
                device="cuda") -> BetaMatrix:
    """CSR (numpy arrays or tensors) -> BetaMatrix on the device."""
    if (r, c) not in SHAPES:
        raise SpcError(-2, "SPC_ERR_UNSUPPORTED_SHAPE", f"({r},{c})")
    rp = _dev(rowptr, torch.int32, device)
    ci = _dev(colidx, torch.int32, device)
    v = _dev(values, dtype, device)
    if ci.numel() == 0:  # the library wants valid pointers even when nothing is read
        ci = torch.zeros(1, dtype=torch.int32, device=device)
    n_rows = rp.numel() - 1
    n_int = (n_rows + r - 1) // r
    L = lib()
    s = stream_ptr()
    brow = torch.empty(n_int + 1, dtype=torch.int32, device=device)
    nb = c_int64()
    check(L.spc_beta_count(r, c, n_rows, n_cols, _ptr(rp), _ptr(ci), _ptr(brow), ctypes.byref(nb), s))
    nb = nb.value
    bcol = torch.empty(nb, dtype=torch.int32, device=device)
    masks = torch.empty(mask_bytes(r, c, nb), dtype=torch.uint8, device=device)
    vout = torch.empty_like(v)
    vin = v if v.numel() else torch.zeros(1, dtype=v.dtype, device=device)
    bcol_p = bcol if nb else torch.zeros(1, dtype=torch.int32, device=device)
    vout_p = vout if v.numel() else torch.zeros(1, dtype=v.dtype, device=device)
    check(L.spc_csr_to_beta(r, c, _dtype_code(v.dtype), n_rows, n_cols, _ptr(rp), _ptr(ci),
                            _ptr(vin), _ptr(brow), _ptr(bcol_p), _ptr(masks), _ptr(vout_p), s))
    return BetaMatrix(r, c, n_rows, n_cols, brow, bcol, masks, vout)


def rcm_order(rowptr, colidx, device="cuda") -> torch.Tensor:
    """Reverse Cuthill-McKee order (perm[new] = old, int32 device tensor) of
    a square CSR pattern."""
    rp = _dev(rowptr, torch.int32, device)
    ci = _dev(colidx, torch.int32, device)
    n, nnz = rp.numel() - 1, ci.numel()
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=device)
    check(lib().spc_rcm_order(n, nnz, _ptr(rp), _ptr(ci) if nnz else None, _ptr(perm), stream_ptr()))
    return perm[:n]


def csr_permute(rowptr, colidx, values, perm, device="cuda"):
    """B = P A P^T (rows and columns renumbered by perm[new] = old) as device
    tensors (rowptr, colidx, values)."""
    rp = _dev(rowptr, torch.int32, device)
    ci = _dev(colidx, torch.int32, device)
    v = _dev(values, None, device)
    pm = _dev(perm, torch.int32, device)
    n, nnz = rp.numel() - 1, ci.numel()
    rp2 = torch.empty(n + 1, dtype=torch.int32, device=device)
    ci2 = torch.empty(nnz, dtype=torch.int32, device=device)
    v2 = torch.empty_like(v)
    check(lib().spc_csr_permute(n, nnz, _ptr(rp), _ptr(ci) if nnz else None, _dtype_code(v.dtype),
                                _ptr(v) if nnz else None, _ptr(pm) if n else None, _ptr(rp2),
                                _ptr(ci2) if nnz else None, _ptr(v2) if nnz else None, stream_ptr()))
    return rp2, ci2, v2


def permute_vector(x: torch.Tensor, perm: torch.Tensor, scatter: bool = False) -> torch.Tensor:
    """scatter False: out[i] = x[perm[i]]; True: out[perm[i]] = x[i]."""
    out = torch.empty_like(x)
    check(lib().spc_permute_vector(x.numel(), _dtype_code(x.dtype), _ptr(perm), _ptr(x), _ptr(out),
                                   int(scatter), stream_ptr()))
    return out


def beta_to_csr(A: BetaMatrix):
    """BetaMatrix -> (rowptr, colidx, values) device tensors."""
    rp = torch.empty(A.n_rows + 1, dtype=torch.int32, device=A.values.device)
    ci = torch.empty(A.nnz, dtype=torch.int32, device=A.values.device)
    v = torch.empty_like(A.values)
    view = A.view()
    check(lib().spc_beta_to_csr(ctypes.byref(view), _ptr(rp), _ptr(ci) if A.nnz else None,
                                _ptr(v) if A.nnz else None, stream_ptr()))
    return rp, ci, v


def spmv(A: BetaMatrix, x: torch.Tensor, y: torch.Tensor | None = None, accumulate: bool = False,
         plan: Plan | None = None) -> torch.Tensor:
    """y = A x (or y += A x) on the device, in A's value type."""
    if x.dtype != A.dtype or x.numel() != A.n_cols or not x.is_contiguous():
        raise ValueError("x must be a contiguous vector of n_cols entries of A's dtype")
    if y is None:
        if accumulate:
            raise ValueError("accumulate needs y")
        y = torch.empty(A.n_rows, dtype=A.dtype, device=x.device)
    elif y.dtype != A.dtype or y.numel() != A.n_rows or not y.is_contiguous():
        raise ValueError("y must be a contiguous vector of n_rows entries of A's dtype")
    plan = plan or A.default_plan()
    view = plan._view
    check(lib().spc_spmv_beta(ctypes.byref(view), plan.handle, _ptr(x), _ptr(y), int(accumulate),
                              stream_ptr()))
    return y


def time_spmv(A: BetaMatrix, plan: Plan | None = None, reps: int = 20, warmup: int = 3) -> float:
    """Average device time (us) of one y = A x launch under the plan."""
    plan = plan or A.default_plan()
    x = torch.zeros(A.n_cols, dtype=A.dtype, device=A.values.device)
    y = torch.empty(A.n_rows, dtype=A.dtype, device=A.values.device)
    us = ctypes.c_float()
    check(lib().spc_time_spmv(ctypes.byref(plan._view), plan.handle, _ptr(x), _ptr(y), warmup, reps,
                              ctypes.byref(us), stream_ptr()))
    return us.value


def autotune(A: BetaMatrix, reps: int = 20, x: torch.Tensor | None = None):
    """Times every candidate plan; returns (best params dict, best us, records)."""
    if x is None:
        x = torch.zeros(A.n_cols, dtype=A.dtype, device=A.values.device)
    y = torch.empty(A.n_rows, dtype=A.dtype, device=A.values.device)
    view = A.view()
    best = PlanParams()
    best_us = ctypes.c_float()
    recs = (TuneRecord * 64)()
    n = c_int32()
    check(lib().spc_autotune(ctypes.byref(view), _ptr(x), _ptr(y), reps, ctypes.byref(best),
                             ctypes.byref(best_us), ctypes.cast(recs, c_void_p), 64, ctypes.byref(n),
                             stream_ptr()))

    records = [dict(_params_dict(recs[i].params), us=recs[i].us, n_tiles=recs[i].n_tiles) for i in range(n.value)]
    return _params_dict(best), best_us.value, records


def _params_dict(p: PlanParams) -> dict:
    d = {"mode": p.mode, "tile_bits": p.tile_bits, "wave_chunks": p.wave_chunks,
         "tile_order": p.tile_order, "pipeline": p.pipeline}
    if p.cu_groups:
        d["cu_groups"] = p.cu_groups
    if p.wave_tiles:
        d["wave_tiles"] = p.wave_tiles
    if p.spmm_path:
        d["spmm_path"] = p.spmm_path
    return d


def plan_from(A: BetaMatrix, params: dict) -> Plan:
    return A.plan(params.get("tile_bits", 0), params.get("tile_order", 0), params.get("mode", 0),
                  params.get("wave_chunks", 0), params.get("pipeline", 0), params.get("cu_groups", 0),
                  params.get("wave_tiles", 0), params.get("spmm_path", 0))


def spmm(A: BetaMatrix, X: torch.Tensor, Y: torch.Tensor | None = None, accumulate: bool = False,
         plan: Plan | None = None) -> torch.Tensor:
    """Y = A X (or Y += A X) for a row-major block X of k <= 16 columns."""
    if X.dim() != 2 or X.shape[0] != A.n_cols or X.dtype != A.dtype or X.stride(1) != 1:
        raise ValueError("X must be n_cols x k, row-major, of A's dtype")
    k = X.shape[1]
    if Y is None:
        if accumulate:
            raise ValueError("accumulate needs Y")
        Y = torch.empty((A.n_rows, k), dtype=A.dtype, device=X.device)
    elif Y.shape != (A.n_rows, k) or Y.dtype != A.dtype or Y.stride(1) != 1:
        raise ValueError("Y must be n_rows x k, row-major, of A's dtype")
    plan = plan or A.default_plan()
    check(lib().spc_spmm_beta(ctypes.byref(plan._view), plan.handle, k, _ptr(X), X.stride(0), _ptr(Y),
                              Y.stride(0), int(accumulate), stream_ptr()))
    return Y


def cg(A: BetaMatrix, B: torch.Tensor, rel_tol: float = 1e-8, max_iter: int = 10000, check_every: int = 10,
       use_graph: bool = True, plan: Plan | None = None):
    """Solve A X = B (k <= 16 columns) by CG from X = 0 on the device.

    Returns (X, iterations per column, relative recurrence residual per
    column, iterations run)."""
    if B.dim() == 1:
        B = B[:, None]
    if B.dim() != 2 or B.shape[0] != A.n_rows or B.dtype != A.dtype:
        raise ValueError("B must be n_rows x k of A's dtype")
    B = B.contiguous()
    k = B.shape[1]
    X = torch.empty_like(B)
    nbytes = int(lib().spc_cg_workspace_bytes(A.n_rows, k, _dtype_code(A.dtype)))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=B.device)
    its = (c_int32 * k)()
    res = (ctypes.c_double * k)()
    tot = c_int32()
    plan = plan or A.default_plan()
    check(lib().spc_cg_solve(ctypes.byref(plan._view), plan.handle, k, _ptr(B), B.stride(0), _ptr(X),
                             X.stride(0), rel_tol, max_iter, check_every, int(use_graph), _ptr(ws), nbytes,
                             ctypes.cast(its, POINTER(c_int32)), ctypes.cast(res, POINTER(ctypes.c_double)),
                             ctypes.byref(tot), stream_ptr()))
    return X, list(its), list(res), tot.value


def matrix_features(rowptr, colidx, n_cols: int, device="cuda"):
    """The 16 selection features of a CSR matrix and its six greedy block
    counts, computed on the device without conversion.
    Returns (float32 numpy array [16], int64 numpy array [6])."""
    import numpy as np
    rp = torch.as_tensor(rowptr, dtype=torch.int32, device=device)
    ci = torch.as_tensor(colidx, dtype=torch.int32, device=device)
    n_rows = rp.numel() - 1
    nnz = ci.numel()
    if nnz == 0:
        ci = torch.zeros(1, dtype=torch.int32, device=device)
    f = (ctypes.c_float * 16)()
    nb = (c_int64 * 6)()
    check(lib().spc_matrix_features(n_rows, n_cols, nnz, _ptr(rp), _ptr(ci), f, nb, stream_ptr()))
    return np.array(list(f), dtype=np.float32), np.array(list(nb), dtype=np.int64)


# ---------------------------------------------------------------------------
# Learned selector (MLP) and interpolation selector

SPMM_AUTO, SPMM_BITS, SPMM_ROWS = 0, 1, 2
MLP_N_PARAMS = 5638
MLP_MAX_BATCH = 64
SEL_INTERP, SEL_MLP = 0, 1
# kernel classes: the six shapes (plan modes 0/1), then the test kernels of
# Algorithm 2 for beta(1,8) and beta(2,4) (plan mode 2)
N_CLASSES = 8
CLASS_TEST_B1X8, CLASS_TEST_B2X4 = 6, 7


def mlp_n_params(n_out: int = 6) -> int:
    """Parameter count of the 16 -> 64 -> 64 -> n_out network."""
    return 64 * 17 + 64 * 65 + n_out * 65


def _mlp_out(params) -> int:
    for k in (6, 8):
        if params.numel() == mlp_n_params(k):
            return k
    raise ValueError(f"params must hold {mlp_n_params(6)} or {mlp_n_params(8)} floats, got {params.numel()}")


def class_shape(k: int) -> int:
    """Shape index (0..5) of kernel class k."""
    s = lib().spc_class_shape(int(k))
    if s < 0:
        raise ValueError(f"no kernel class {k}")
    return s


def class_mode(k: int) -> int:
    """Plan mode of kernel class k: 2 for the test classes, -1 for a shape's own kernels."""
    return int(lib().spc_class_mode(int(k)))


def _f32_cuda(t, shape=None):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return t


def _i32_host(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(POINTER(c_int32))


def mlp_standardizer(X: torch.Tensor):
    """(mu, sd) of the n x 16 feature rows, on the device."""
    n = X.shape[0]
    _f32_cuda(X, (n, 16))
    mu = torch.empty(16, dtype=torch.float32, device=X.device)
    sd = torch.empty(16, dtype=torch.float32, device=X.device)
    check(lib().spc_mlp_standardizer(_ptr(X), n, _ptr(mu), _ptr(sd), stream_ptr()))
    return mu, sd


def mlp_targets(times: torch.Tensor) -> torch.Tensor:
    """tau = log2(t / row minimum) of n x K times (K = 6 or 8)."""
    n = times.shape[0]
    k = times.shape[1] if times.dim() == 2 else 0
    _f32_cuda(times, (n, k))
    tau = torch.empty_like(times)
    check(lib().spc_mlp_targets(_ptr(times), n, k, _ptr(tau), stream_ptr()))
    return tau


def mlp_loss_grad(params, mu, sd, X, tau, rows):
    """Loss and gradient of one batch (rows: host indices into X/tau)."""
    n = X.shape[0]
    k = _mlp_out(params)
    for t, shp in ((params, (mlp_n_params(k),)), (mu, (16,)), (sd, (16,)), (X, (n, 16)), (tau, (n, k))):
        _f32_cuda(t, shp)
    r, rp = _i32_host(rows)
    grad = torch.empty(mlp_n_params(k), dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    check(lib().spc_mlp_loss_grad(_ptr(params), _ptr(mu), _ptr(sd), _ptr(X), _ptr(tau), n, k, rp, r.size,
                                  _ptr(grad), _ptr(loss), stream_ptr()))
    return float(loss.item()), grad


def mlp_train(params, adam_m, adam_v, step0: int, lr: float, mu, sd, X, tau, order, batch: int):
    """Adam steps over batches order[s*batch:(s+1)*batch] (host indices);
    params and moments are updated in place. Returns the per-step losses."""
    n = X.shape[0]
    k = _mlp_out(params)
    npar = mlp_n_params(k)
    for t, shp in ((params, (npar,)), (adam_m, (npar,)), (adam_v, (npar,)),
                   (mu, (16,)), (sd, (16,)), (X, (n, 16)), (tau, (n, k))):
        _f32_cuda(t, shp)
    o, op = _i32_host(order)
    steps = o.size // batch
    losses = torch.empty(max(1, steps), dtype=torch.float32, device=X.device)
    check(lib().spc_mlp_train(_ptr(params), _ptr(adam_m), _ptr(adam_v), step0, lr, _ptr(mu), _ptr(sd), _ptr(X),
                              _ptr(tau), n, k, op, steps, batch, _ptr(losses), stream_ptr()))
    return losses[:steps]


def mlp_infer(params, mu, sd, X):
    """(scores n x K, choice n) of the network (K outputs, 6 or 8) for n
    feature rows."""
    n = X.shape[0]
    k = _mlp_out(params)
    for t, shp in ((params, (mlp_n_params(k),)), (mu, (16,)), (sd, (16,)), (X, (n, 16))):
        _f32_cuda(t, shp)
    scores = torch.empty((n, k), dtype=torch.float32, device=X.device)
    choice = torch.empty(n, dtype=torch.int32, device=X.device)
    check(lib().spc_mlp_infer(_ptr(params), _ptr(mu), _ptr(sd), _ptr(X), n, k, _ptr(scores), _ptr(choice),
                              stream_ptr()))
    return scores, choice


class Selector:
    """Library-owned selector: interpolation fit and/or a trained network."""

    def __init__(self):
        h = c_void_p()
        check(lib().spc_selector_create(ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.spc_selector_destroy(h)
            self.handle = None

    def fit_interp(self, avg, speed, degree: int = 3):
        """Per-class polynomial fit; avg and speed are n x K (K = 6 shapes
        or 8 kernel classes; the Avg of a test class is its shape's)."""
        import numpy as np
        a = np.ascontiguousarray(avg, dtype=np.float64)
        v = np.ascontiguousarray(speed, dtype=np.float64)
        if a.ndim != 2 or a.shape[1] not in (6, 8) or v.shape != a.shape:
            raise ValueError("avg and speed must be n x 6 or n x 8")
        check(lib().spc_selector_fit_interp(self.handle, a.shape[0], a.shape[1],
                                            a.ctypes.data_as(POINTER(ctypes.c_double)),
                                            v.ctypes.data_as(POINTER(ctypes.c_double)), degree))
        return self

    def interp_coeffs(self):
        import numpy as np
        c = np.zeros((N_CLASSES, 4))
        lo = np.zeros(N_CLASSES)
        hi = np.zeros(N_CLASSES)
        k = c_int32()
        dp = POINTER(ctypes.c_double)
        check(lib().spc_selector_interp_coeffs(self.handle, c.ctypes.data_as(dp), lo.ctypes.data_as(dp),
                                               hi.ctypes.data_as(dp), ctypes.byref(k)))
        k = int(k.value)
        return c[:k], lo[:k], hi[:k]

    def n_classes(self, method: int = SEL_MLP) -> int:
        return int(lib().spc_selector_n_classes(self.handle, method))

    def set_mlp(self, params, mu, sd):
        import numpy as np
        fp = POINTER(ctypes.c_float)
        p = np.ascontiguousarray(params, dtype=np.float32)
        m = np.ascontiguousarray(mu, dtype=np.float32)
        s_ = np.ascontiguousarray(sd, dtype=np.float32)
        k = 8 if p.size == mlp_n_params(8) else 6
        if p.size != mlp_n_params(k) or m.size != 16 or s_.size != 16:
            raise ValueError(f"params must hold {mlp_n_params(6)} or {mlp_n_params(8)} floats, mu and sd 16 each")
        check(lib().spc_selector_set_mlp(self.handle, k, p.ctypes.data_as(fp), m.ctypes.data_as(fp),
                                         s_.ctypes.data_as(fp)))
        return self

    def fit_interp2d(self, avg, log2_share, speed, deg_avg: int = 3, deg_share: int = 2):
        """2-D fit of speed against (Avg, log2 of the compute-unit share)."""
        import numpy as np
        a = np.ascontiguousarray(avg, dtype=np.float64)
        u = np.ascontiguousarray(log2_share, dtype=np.float64)
        v = np.ascontiguousarray(speed, dtype=np.float64)
        if a.ndim != 2 or a.shape[1] != 6 or v.shape != a.shape or u.shape != (a.shape[0],):
            raise ValueError("avg and speed must be n x 6, log2_share n")
        dp = POINTER(ctypes.c_double)
        check(lib().spc_selector_fit_interp2d(self.handle, a.shape[0], a.ctypes.data_as(dp), u.ctypes.data_as(dp),
                                              v.ctypes.data_as(dp), deg_avg, deg_share))
        return self

    def interp2d_coeffs(self):
        import numpy as np
        c = np.zeros((6, 4, 3))
        lo = np.zeros(6)
        hi = np.zeros(6)
        ur = np.zeros(2)
        dp = POINTER(ctypes.c_double)
        check(lib().spc_selector_interp2d_coeffs(self.handle, c.ctypes.data_as(dp), lo.ctypes.data_as(dp),
                                                 hi.ctypes.data_as(dp), ur.ctypes.data_as(dp)))
        return c, lo, hi, ur

    def select_at(self, features, cu_share: float):
        """(shape index, predicted GFlop/s[6]) at a share of the compute units."""
        import numpy as np
        f = np.ascontiguousarray(features, dtype=np.float32)
        out = c_int32()
        sc = (ctypes.c_float * 6)()
        check(lib().spc_select_kernel_at(self.handle, f.ctypes.data_as(POINTER(ctypes.c_float)), float(cu_share),
                                         ctypes.byref(out), sc))
        return int(out.value), np.array(list(sc), dtype=np.float32)

    def select(self, features, method: int = SEL_MLP):
        """(kernel class, scores[K]) for one host feature vector; K is the
        model's class count (6: shapes, 8: shapes and the test kernels)."""
        import numpy as np
        f = np.ascontiguousarray(features, dtype=np.float32)
        if f.size != 16:
            raise ValueError("features must hold 16 floats")
        out = c_int32()
        sc = (ctypes.c_float * N_CLASSES)()
        check(lib().spc_select_kernel(self.handle, f.ctypes.data_as(POINTER(ctypes.c_float)), method,
                                      ctypes.byref(out), sc, stream_ptr() if method == SEL_MLP else None))
        k = self.n_classes(method)
        return int(out.value), np.array(list(sc)[:k], dtype=np.float32)


class CUStream:
    """A HIP stream restricted to n_cus compute units, usable as a torch
    stream (torch.cuda.ExternalStream) for this library's calls."""

    def __init__(self, n_cus: int):
        h = c_void_p()
        check(lib().spc_stream_create_cu(int(n_cus), ctypes.byref(h)))
        self.handle = h
        self.n_cus = int(n_cus)
        self.stream = torch.cuda.ExternalStream(h.value)

    def close(self):
        if self.handle is not None and self.handle.value:
            self.stream.synchronize()
            check(lib().spc_stream_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_cu_count() -> int:
    return int(lib().spc_device_cu_count())


def _plan_params(d: dict) -> PlanParams:
    return PlanParams(d.get("tile_bits", 0), d.get("tile_order", 0), d.get("mode", 0), d.get("wave_chunks", 0),
                      d.get("pipeline", 0), d.get("cu_groups", 0), d.get("wave_tiles", 0), d.get("spmm_path", 0))


class Batch:
    """Products of many BetaMatrix objects, one launch per group of matrices
    that share (mode, shape, chunk count) (library-owned batch).

    params: None (each matrix's default parameters), one dict for all
    matrices, or a list of one dict per matrix (keys as plan_from takes;
    mode 0, 2, 3 or 4). wave_chunks alone gives every matrix mode 0 with
    that chunk count."""

    def __init__(self, mats: list, wave_chunks: int | None = None, params=None):
        if not mats:
            raise ValueError("need at least one matrix")
        self.mats = list(mats)
        self._views = (BetaView * len(mats))(*[m.view() for m in mats])
        if params is None and wave_chunks is not None:
            params = {"mode": 0, "wave_chunks": wave_chunks}
        if params is None:
            arr, n = None, 0
        elif isinstance(params, dict):
            arr, n = (PlanParams * 1)(_plan_params(params)), 1
        else:
            if len(params) != len(mats):
                raise ValueError("one parameter set per matrix")
            arr, n = (PlanParams * len(mats))(*[_plan_params(d) for d in params]), len(mats)
        h = c_void_p()
        check(lib().spc_batch_create(len(mats), self._views, arr, n, ctypes.byref(h), stream_ptr()))
        self.handle = h
        self._xs = self._ys = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.spc_batch_destroy(h)
            self.handle = None

    def info(self) -> dict:
        nt, nl, ss, ng = c_int64(), c_int64(), c_int32(), c_int32()
        check(lib().spc_batch_info(self.handle, ctypes.byref(nt), ctypes.byref(nl), ctypes.byref(ss),
                                   ctypes.byref(ng)))
        return {"n_tiles": nt.value, "n_long": nl.value, "single_shape": ss.value, "n_groups": ng.value}

    def set_kernel(self, general: bool):
        """general=True runs the whole list as one launch of the
        shape-switching kernel (every matrix in mode 0, one chunk count)."""
        check(lib().spc_batch_set_kernel(self.handle, int(general)))
        return self

    def set_vectors(self, xs: list, ys: list):
        if len(xs) != len(self.mats) or len(ys) != len(self.mats):
            raise ValueError("one x and one y per matrix")
        for A, x, y in zip(self.mats, xs, ys):
            if x.numel() != A.n_cols or y.numel() != A.n_rows or x.dtype != A.dtype or y.dtype != A.dtype \
                    or not x.is_contiguous() or not y.is_contiguous():
                raise ValueError("x_i / y_i must be contiguous vectors of A_i's sizes and dtype")
        n = len(self.mats)
        xa = (c_void_p * n)(*[x.data_ptr() for x in xs])
        ya = (c_void_p * n)(*[y.data_ptr() for y in ys])
        check(lib().spc_batch_set_vectors(self.handle, xa, ya))
        self._xs, self._ys = list(xs), list(ys)  # keep them alive
        return self

    def run(self, accumulate: bool = False, grid_blocks: int = 0, use_graph: bool = False):
        check(lib().spc_spmv_batched(self.handle, int(accumulate), grid_blocks, int(use_graph), stream_ptr()))
