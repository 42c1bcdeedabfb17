"""ctypes binding of librorbk.so (include/rorbk.h).

Argument marshalling only: torch tensors supply device memory and the stream;
every step of the method runs in the HIP library.  Importing works without a
GPU (so the ABI can be inspected), but any call that needs the device fails
loudly when the library or the device is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librorbk.so")

# status codes and flags (include/rorbk.h)
RORBK_OK = 0
RORBK_ERR_INVALID_ARG = 1
RORBK_ERR_OOM = 2
RORBK_ERR_HIP = 3
RORBK_ERR_NOT_SPD = 4
RORBK_ERR_NONFINITE = 5
RORBK_ERR_NOT_RECORDED = 6
RORBK_ERR_UNSUPPORTED = 7
RORBK_MAX_BLOCK_ROWS = 160
RORBK_MAX_BIG_BLOCK_ROWS = 2048
RORBK_DENSE, RORBK_CSR = 0, 1
RORBK_F64, RORBK_F32, RORBK_BF16 = 0, 1, 2
RORBK_REFINE, RORBK_RECORD, RORBK_REPLAY, RORBK_CHECKPOINT = 1, 2, 4, 8
RORBK_PROFILE = 16
RORBK_NOALLOC_SCRATCH_BYTES = 16777216

EXPORTS = [
    "ror_bk_partition", "ror_bk_setup", "ror_bk_solve", "ror_bk_backward", "ror_bk_destroy",
    "ror_bk_get_sizes", "ror_bk_get_setup", "ror_bk_set_proposal",
    "ror_bk_get_block_inverse", "ror_bk_get_form", "ror_bk_sample", "ror_bk_topk", "ror_bk_residual",
    "ror_bk_residual_noalloc", "ror_bk_get_record", "ror_bk_set_replay", "ror_bk_set_refine",
    "ror_bk_get_profile", "ror_bk_initial_solution", "ror_bk_fabgmres", "ror_bk_error_string",
    "ror_bk_last_error_message",
]


class RorBkError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        msg = f"{what}: {_ERR.get(code, 'status ' + str(code))}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)
        self.code = code


_ERR = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "HIP runtime error",
        4: "block Gram not positive definite", 5: "non-finite residual",
        6: "no recorded solve", 7: "unsupported configuration"}


class rorbk_matrix(C.Structure):
    _fields_ = [("format", C.c_int32), ("dtype", C.c_int32), ("m", C.c_int64),
                ("n", C.c_int64), ("ld", C.c_int64), ("values", C.c_void_p),
                ("rowptr", C.c_void_p), ("colidx", C.c_void_p), ("nnz", C.c_int64),
                ("values_f64", C.c_void_p)]


class rorbk_info(C.Structure):
    _fields_ = [("iters", C.c_int64), ("rrn", C.c_double), ("converged", C.c_int32),
                ("n_refine", C.c_int32), ("t_solve_s", C.c_double), ("t_setup_s", C.c_double),
                ("rrn_test", C.c_double)]


_lib = None


def lib():
    """Load librorbk.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with paper_2510_02156_amd/build.py "
                "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        sig = {
            "ror_bk_partition": (C.c_int, [I64, I64, P, P]),
            "ror_bk_setup": (C.c_int, [C.POINTER(rorbk_matrix), I64, D, P, C.POINTER(P)]),
            "ror_bk_solve": (C.c_int, [P, P, P, C.c_uint64, D, I64, I64, C.c_uint32, I64,
                                       C.POINTER(rorbk_info)]),
            "ror_bk_backward": (C.c_int, [P, P, P, P]),
            "ror_bk_destroy": (C.c_int, [P]),
            "ror_bk_get_sizes": (C.c_int, [P, P, P, P]),
            "ror_bk_get_setup": (C.c_int, [P, P, P, P, P]),
            "ror_bk_set_proposal": (C.c_int, [P, P]),
            "ror_bk_get_block_inverse": (C.c_int, [P, I64, P]),
            "ror_bk_get_form": (C.c_int, [P, P]),
            "ror_bk_sample": (C.c_int, [P, C.c_uint64, I64, I64, P]),
            "ror_bk_topk": (C.c_int, [P, P, I32, P]),
            "ror_bk_residual": (C.c_int, [P, P, P, P, P, I32, I32, P]),
            "ror_bk_residual_noalloc": (C.c_int, [C.POINTER(rorbk_matrix), I64, P, P, P, P, P,
                                                  I32, P]),
            "ror_bk_get_record": (C.c_int, [P, P, P, P, P]),
            "ror_bk_set_replay": (C.c_int, [P, P, P, I64]),
            "ror_bk_set_refine": (C.c_int, [P, I64, D]),
            "ror_bk_get_profile": (C.c_int, [P, P]),
            "ror_bk_initial_solution": (C.c_int, [P, P, P, I32, P]),
            "ror_bk_fabgmres": (C.c_int, [P, P, P, C.c_uint64, D, I64, I64, D,
                                          C.POINTER(rorbk_info)]),
            "ror_bk_error_string": (C.c_char_p, [C.c_int]),
            "ror_bk_last_error_message": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != RORBK_OK:
        detail = lib().ror_bk_last_error_message().decode(errors="replace")
        raise RorBkError(rc, what, detail)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    return C.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


_DT = {"float64": RORBK_F64, "float32": RORBK_F32, "bfloat16": RORBK_BF16}


def _dtype_code(t) -> int:
    name = str(t.dtype).replace("torch.", "")
    if name not in _DT:
        raise ValueError(f"unsupported matrix dtype {t.dtype}")
    return _DT[name]


# ------------------------------------------------------------ raw entry points

def ror_bk_partition(m: int, block_rows: int) -> np.ndarray:
    """The k+1 block offsets (host computation in the library, no device)."""
    k = C.c_int64()
    _check(lib().ror_bk_partition(int(m), int(block_rows), None, C.byref(k)),
           "ror_bk_partition")
    off = np.zeros(k.value + 1, dtype=np.int64)
    _check(lib().ror_bk_partition(int(m), int(block_rows), _np_ptr(off), C.byref(k)),
           "ror_bk_partition")
    return off


def ror_bk_setup(A=None, block_rows: int = 1, lam: float = 0.0, stream=None, *,
                 rowptr=None, colidx=None, values=None, shape=None, A64=None):
    """Set up a handle.  Dense: ``A`` a 2-D CUDA tensor with unit column stride
    (row stride = ld).  CSR: ``rowptr`` (int64), ``colidx`` (int32),
    ``values`` and ``shape``.  ``A64``: optional FP64 master copy (same layout).
    Returns (handle, descriptor); keep the tensors alive while the handle lives."""
    d = matrix_descriptor(A, rowptr=rowptr, colidx=colidx, values=values, shape=shape, A64=A64)
    h = C.c_void_p()
    _check(lib().ror_bk_setup(C.byref(d), int(block_rows), float(lam), _stream_ptr(stream),
                              C.byref(h)), "ror_bk_setup")
    return h, d


def matrix_descriptor(A=None, *, rowptr=None, colidx=None, values=None, shape=None, A64=None):
    """rorbk_matrix for a dense 2-D tensor ``A`` (unit column stride) or CSR
    arrays; the tensors must outlive every use of the descriptor."""
    d = rorbk_matrix()
    if A is not None:
        if A.dim() != 2 or A.stride(1) != 1:
            raise ValueError("dense A must be 2-D with unit column stride")
        d.format = RORBK_DENSE
        d.dtype = _dtype_code(A)
        d.m, d.n = A.shape
        d.ld = A.stride(0)
        d.values = A.data_ptr()
        d.nnz = 0
    else:
        d.format = RORBK_CSR
        d.dtype = _dtype_code(values)
        d.m, d.n = shape
        d.ld = shape[1]
        d.values = values.data_ptr()
        d.rowptr = rowptr.data_ptr()
        d.colidx = colidx.data_ptr()
        d.nnz = values.numel()
    d.values_f64 = A64.data_ptr() if A64 is not None else None
    return d


def ror_bk_solve(h, b, x, seed: int, tol: float, max_iters: int, start_iter: int = 0,
                 flags: int = 0, checkpoint_every: int = 0) -> dict:
    info = rorbk_info()
    _check(lib().ror_bk_solve(h, _dev_ptr(b), _dev_ptr(x), seed & ((1 << 64) - 1), float(tol),
                              int(max_iters), int(start_iter), int(flags),
                              int(checkpoint_every), C.byref(info)), "ror_bk_solve")
    return {"iters": info.iters, "rrn": info.rrn, "converged": bool(info.converged),
            "n_refine": info.n_refine, "t_solve_s": info.t_solve_s,
            "t_setup_s": info.t_setup_s, "rrn_test": info.rrn_test}


def ror_bk_backward(h, grad_x, grad_b, grad_x0):
    _check(lib().ror_bk_backward(h, _dev_ptr(grad_x), _dev_ptr(grad_b), _dev_ptr(grad_x0)),
           "ror_bk_backward")


def ror_bk_destroy(h):
    if h:
        _check(lib().ror_bk_destroy(h), "ror_bk_destroy")


def ror_bk_get_sizes(h):
    k, K, bmax = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().ror_bk_get_sizes(h, C.byref(k), C.byref(K), C.byref(bmax)), "ror_bk_get_sizes")
    return k.value, K.value, bmax.value


def ror_bk_get_setup(h):
    k, _, _ = ror_bk_get_sizes(h)
    off = np.zeros(k + 1, dtype=np.int64)
    S, pbar, W = np.zeros(k), np.zeros(k), np.zeros(k)
    _check(lib().ror_bk_get_setup(h, _np_ptr(off), _np_ptr(S), _np_ptr(pbar), _np_ptr(W)),
           "ror_bk_get_setup")
    return {"offsets": off, "S": S, "pbar": pbar, "W": W}


def ror_bk_set_proposal(h, W):
    W = np.ascontiguousarray(W, dtype=np.float64)
    _check(lib().ror_bk_set_proposal(h, _np_ptr(W)), "ror_bk_set_proposal")


def ror_bk_get_form(h) -> int:
    col = C.c_int32()
    _check(lib().ror_bk_get_form(h, C.byref(col)), "ror_bk_get_form")
    return col.value


def ror_bk_get_block_inverse(h, t: int, rows: int):
    out = np.zeros((rows, rows))
    _check(lib().ror_bk_get_block_inverse(h, int(t), _np_ptr(out)), "ror_bk_get_block_inverse")
    return out


def ror_bk_sample(h, seed: int, j0: int, count: int):
    out = np.zeros(3 * count, dtype=np.int32)
    _check(lib().ror_bk_sample(h, seed & ((1 << 64) - 1), int(j0), int(count), _np_ptr(out)),
           "ror_bk_sample")
    return out


def ror_bk_topk(h, r, idx):
    vec_f32 = 1 if str(r.dtype) == "torch.float32" else 0
    _check(lib().ror_bk_topk(h, _dev_ptr(r), vec_f32, _dev_ptr(idx)), "ror_bk_topk")


def ror_bk_residual(h, b, x, r, block_norm2=None, use_f64_master: bool = False) -> float:
    vec_f32 = 1 if str(b.dtype) == "torch.float32" else 0
    rrn = C.c_double()
    _check(lib().ror_bk_residual(h, _dev_ptr(b), _dev_ptr(x), _dev_ptr(r), _dev_ptr(block_norm2),
                                 vec_f32, int(bool(use_f64_master)), C.byref(rrn)),
           "ror_bk_residual")
    return rrn.value


def ror_bk_residual_noalloc(desc, block_rows: int, b, x, r, block_norm2=None, rrn=None,
                            stream=None):
    """Enqueue the handle-free, allocation-free residual pass (device outputs
    r, block_norm2, rrn; nothing is synchronised or allocated here)."""
    vec_f32 = 1 if str(b.dtype) == "torch.float32" else 0
    _check(lib().ror_bk_residual_noalloc(C.byref(desc), int(block_rows), _dev_ptr(b), _dev_ptr(x),
                                         _dev_ptr(r), _dev_ptr(block_norm2), _dev_ptr(rrn),
                                         vec_f32, _stream_ptr(stream)),
           "ror_bk_residual_noalloc")


def ror_bk_get_record(h, K: int):
    it = C.c_int64()
    _check(lib().ror_bk_get_record(h, None, None, None, C.byref(it)), "ror_bk_get_record")
    n = it.value
    tau = np.zeros(3 * n, dtype=np.int32)
    rrn = np.zeros(n)
    I = np.zeros(n * K, dtype=np.int32)
    _check(lib().ror_bk_get_record(h, _np_ptr(tau), None, _np_ptr(rrn), C.byref(it)),
           "ror_bk_get_record")
    got_I = lib().ror_bk_get_record(h, None, _np_ptr(I), None, C.byref(it))
    return {"iters": n, "tau": tau, "rrn": rrn,
            "I": I.reshape(n, K) if got_I == RORBK_OK else None}


def ror_bk_initial_solution(h, b, x0) -> float:
    """Algorithm 2's x0 into x0 (vector type of b); returns the coefficient."""
    vec_f32 = 1 if str(b.dtype) == "torch.float32" else 0
    coef = C.c_double()
    _check(lib().ror_bk_initial_solution(h, _dev_ptr(b), _dev_ptr(x0), vec_f32, C.byref(coef)),
           "ror_bk_initial_solution")
    return coef.value


def ror_bk_fabgmres(h, b, x, seed: int, tol: float, max_outer: int, inner_iters: int,
                    eta: float) -> dict:
    info = rorbk_info()
    _check(lib().ror_bk_fabgmres(h, _dev_ptr(b), _dev_ptr(x), seed & ((1 << 64) - 1), float(tol),
                                 int(max_outer), int(inner_iters), float(eta), C.byref(info)),
           "ror_bk_fabgmres")
    return {"inner_iters": info.iters, "outer": info.n_refine, "converged": bool(info.converged),
            "rrn": info.rrn, "t_setup_s": info.t_setup_s}


def ror_bk_set_replay(h, tau, I, iters: int):
    tau = np.ascontiguousarray(tau, dtype=np.int32).reshape(-1)
    I = np.ascontiguousarray(I, dtype=np.int32).reshape(-1)
    _check(lib().ror_bk_set_replay(h, _np_ptr(tau), _np_ptr(I), int(iters)), "ror_bk_set_replay")


def ror_bk_set_refine(h, inner_iters: int, eta: float):
    _check(lib().ror_bk_set_refine(h, int(inner_iters), float(eta)), "ror_bk_set_refine")


def ror_bk_get_profile(h) -> dict:
    out = np.zeros(4)
    _check(lib().ror_bk_get_profile(h, _np_ptr(out)), "ror_bk_get_profile")
    return {"inner_ms": out[0], "inner_n": int(out[1]), "outer_ms": out[2],
            "outer_n": int(out[3])}


def ror_bk_error_string(code: int) -> str:
    return lib().ror_bk_error_string(int(code)).decode()
