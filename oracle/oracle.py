"""ctypes front end of the C oracle (oracle/rorbk_oracle.c).

Test infrastructure: arrays in, arrays out, all FP64 on the host.  A matrix is
passed either as a 2-D numpy array (dense) or as a workload dict from
``workloads.make`` (``format`` "dense" with ``A``, or "csr" with ``rowptr``,
``colidx``, ``val``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

ORC_OK, ORC_ERR_ARG, ORC_ERR_OOM, ORC_ERR_NOT_SPD, ORC_ERR_NONFINITE = 0, 1, 2, 4, 5


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


class _Mat(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("csr", C.c_int32),
                ("pad_", C.c_int32), ("a", C.c_void_p), ("ld", C.c_int64),
                ("rowptr", C.c_void_p), ("colidx", C.c_void_p),
                ("val", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_num_blocks.restype = C.c_int64
        L.orc_num_blocks.argtypes = [C.c_int64, C.c_int64]
        L.orc_partition.restype = None
        L.orc_partition.argtypes = [C.c_int64, C.c_int64, P]
        L.orc_cosine_rowsums.restype = C.c_int
        L.orc_cosine_rowsums.argtypes = [P, C.c_int64, P, C.c_int64, C.c_int64, P]
        L.orc_proposal.restype = None
        L.orc_proposal.argtypes = [P, C.c_int64, C.c_int64, P, P]
        L.orc_splitmix64_word.restype = C.c_uint64
        L.orc_splitmix64_word.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_sample.restype = C.c_int32
        L.orc_sample.argtypes = [C.c_uint64, C.c_int64, C.c_int32, P, C.c_int64]
        L.orc_cholesky.restype = C.c_int
        L.orc_cholesky.argtypes = [P, C.c_int64]
        L.orc_chol_solve.restype = None
        L.orc_chol_solve.argtypes = [P, C.c_int64, P, P]
        L.orc_block_factor.restype = C.c_int
        L.orc_block_factor.argtypes = [P, P, C.c_int64, C.c_double, P]
        L.orc_apply_block.restype = C.c_int
        L.orc_apply_block.argtypes = [P, P, C.c_int64, C.c_double, P, P]
        L.orc_residual.restype = None
        L.orc_residual.argtypes = [P, P, P, P]
        L.orc_topk.restype = C.c_int
        L.orc_topk.argtypes = [P, C.c_int64, C.c_int64, P]
        L.orc_solve.restype = C.c_int
        L.orc_solve.argtypes = [P, C.c_int64, C.c_double, P, P, C.c_uint64,
                                C.c_double, C.c_int64, C.c_int64, P, P, P,
                                P, P, P, P, P, P]
        L.orc_backward.restype = C.c_int
        L.orc_backward.argtypes = [P, C.c_int64, C.c_double, P, P, C.c_int64,
                                   C.c_int32, P, P]
        L.orc_num_threads.restype = C.c_int
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_fabgmres.restype = C.c_int
        L.orc_fabgmres.argtypes = [P, C.c_int64, C.c_double, P, P, C.c_uint64, C.c_double,
                                   C.c_int64, C.c_int64, C.c_double, P, P, P, P, P]
        L.orc_initial_solution.restype = C.c_int
        L.orc_initial_solution.argtypes = [P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Matrix:
    """Keeps the numpy buffers alive while the C struct points at them."""

    def __init__(self, A):
        if isinstance(A, dict):
            if A["format"] == "csr":
                self.rowptr = np.ascontiguousarray(A["rowptr"], dtype=np.int64)
                self.colidx = np.ascontiguousarray(A["colidx"], dtype=np.int32)
                self.val = _f64(A["val"])
                self.m = int(A["m"])
                self.n = int(A["n"])
                self.csr = True
            else:
                A = A["A"]
        if not isinstance(A, dict):
            a = _f64(A)
            assert a.ndim == 2
            self.a = a
            self.m, self.n = a.shape
            self.csr = False
        s = _Mat()
        s.m, s.n, s.csr = self.m, self.n, int(self.csr)
        if self.csr:
            s.a, s.ld = None, 0
            s.rowptr, s.colidx, s.val = _p(self.rowptr), _p(self.colidx), _p(self.val)
        else:
            s.a, s.ld = _p(self.a), self.n
            s.rowptr = s.colidx = s.val = None
        self.s = s

    @property
    def ptr(self):
        return C.byref(self.s)

    def dense(self) -> np.ndarray:
        if not self.csr:
            return self.a
        d = np.zeros((self.m, self.n))
        for i in range(self.m):
            lo, hi = self.rowptr[i], self.rowptr[i + 1]
            d[i, self.colidx[lo:hi]] = self.val[lo:hi]
        return d


def _mat(A) -> Matrix:
    return A if isinstance(A, Matrix) else Matrix(A)


def num_blocks(m: int, block_rows: int) -> int:
    return int(lib().orc_num_blocks(m, block_rows))


def partition(m: int, block_rows: int) -> np.ndarray:
    k = num_blocks(m, block_rows)
    if k <= 0:
        raise OracleError(ORC_ERR_ARG, "partition")
    off = np.zeros(k + 1, dtype=np.int64)
    lib().orc_partition(m, k, _p(off))
    return off


def cosine_rowsums(A, block_rows: int, t_lo: int = 0, t_hi: int | None = None):
    M = _mat(A)
    off = partition(M.m, block_rows)
    k = len(off) - 1
    t_hi = k if t_hi is None else t_hi
    S = np.zeros(t_hi - t_lo)
    rc = lib().orc_cosine_rowsums(M.ptr, k, _p(off), t_lo, t_hi, _p(S))
    if rc:
        raise OracleError(rc, "cosine_rowsums")
    return S


def proposal(S: np.ndarray, n: int):
    S = _f64(S)
    pbar = np.zeros_like(S)
    W = np.zeros_like(S)
    lib().orc_proposal(_p(S), len(S), n, _p(pbar), _p(W))
    return pbar, W


def splitmix64_word(seed: int, c: int) -> int:
    return int(lib().orc_splitmix64_word(seed, c))


def sample(seed: int, j: int, l: int, W: np.ndarray) -> int:
    W = _f64(W)
    return int(lib().orc_sample(seed, j, l, _p(W), len(W)))


def sample_many(seed: int, j0: int, iters: int, W: np.ndarray) -> np.ndarray:
    W = _f64(W)
    out = np.empty(3 * iters, dtype=np.int32)
    L = lib()
    for it in range(iters):
        for l in (1, 2, 3):
            out[3 * it + l - 1] = L.orc_sample(seed, j0 + it, l, _p(W), len(W))
    return out


def cholesky(G: np.ndarray) -> np.ndarray:
    L = _f64(G).copy()
    rc = lib().orc_cholesky(_p(L), L.shape[0])
    if rc:
        raise OracleError(rc, "cholesky")
    return np.tril(L)


def chol_solve(L: np.ndarray, r: np.ndarray) -> np.ndarray:
    L = _f64(L)
    r = _f64(r)
    y = np.zeros_like(r)
    lib().orc_chol_solve(_p(L), L.shape[0], _p(r), _p(y))
    return y


def block_factor(A, rows, mu: float) -> np.ndarray:
    M = _mat(A)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    K = len(rows)
    L = np.zeros((K, K))
    rc = lib().orc_block_factor(M.ptr, _p(rows), K, mu, _p(L))
    if rc:
        raise OracleError(rc, "block_factor")
    return np.tril(L)


def apply_block(A, rows, mu: float, b, x) -> np.ndarray:
    """One regularised block update of x on the given rows; returns the new x."""
    M = _mat(A)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    b = _f64(b)
    x = _f64(x).copy()
    rc = lib().orc_apply_block(M.ptr, _p(rows), len(rows), mu, _p(b), _p(x))
    if rc:
        raise OracleError(rc, "apply_block")
    return x


def residual(A, b, x) -> np.ndarray:
    M = _mat(A)
    b, x = _f64(b), _f64(x)
    r = np.zeros(M.m)
    lib().orc_residual(M.ptr, _p(b), _p(x), _p(r))
    return r


def topk(r: np.ndarray, K: int) -> np.ndarray:
    r = _f64(r)
    idx = np.zeros(K, dtype=np.int32)
    rc = lib().orc_topk(_p(r), len(r), K, _p(idx))
    if rc:
        raise OracleError(rc, "topk")
    return idx


def solve(A, block_rows: int, mu: float, b, x0=None, seed: int = 0,
          tol: float = 0.0, max_iters: int = 100, start_iter: int = 0,
          W=None, replay_tau=None, replay_I=None, record: bool = True) -> dict:
    """Algorithm 1 on the host in FP64.  Returns x, iterations, convergence,
    the last RRN and (with ``record``) the recorded tau, I and RRN history."""
    M = _mat(A)
    k = num_blocks(M.m, block_rows)
    if k <= 0:
        raise OracleError(ORC_ERR_ARG, "solve")
    K = M.m // k
    b = _f64(b)
    x = np.zeros(M.n) if x0 is None else _f64(x0).copy()
    Wa = None if W is None else _f64(W)
    rt = None if replay_tau is None else np.ascontiguousarray(replay_tau, dtype=np.int32)
    rI = None if replay_I is None else np.ascontiguousarray(replay_I, dtype=np.int32)
    tau = np.zeros(3 * max_iters, dtype=np.int32) if record else None
    Is = np.zeros(max_iters * K, dtype=np.int32) if record else None
    rr = np.zeros(max_iters) if record else None
    ints = np.zeros(2, dtype=np.int64)
    rrn = np.zeros(1)
    times = np.zeros(2)
    rc = lib().orc_solve(M.ptr, block_rows, mu, _p(b), _p(x), seed & ((1 << 64) - 1),
                         tol, max_iters, start_iter, _p(Wa), _p(rt), _p(rI),
                         _p(tau), _p(Is), _p(rr), _p(ints), _p(rrn), _p(times))
    if rc:
        raise OracleError(rc, "solve")
    it = int(ints[0])
    out = {"x": x, "iters": it, "converged": bool(ints[1]), "rrn": float(rrn[0]),
           "K": K, "k": k, "t_setup_s": float(times[0]), "t_iter_s": float(times[1])}
    if record:
        out["tau"] = tau[: 3 * it].copy()
        out["I"] = Is[: it * K].reshape(it, K).copy()
        out["rrn_hist"] = rr[:it].copy()
    return out


def backward(A, block_rows: int, mu: float, tau, Isets, iters: int,
             converged: bool, grad_x):
    """dL/db and dL/dx0 given dL/dx_final and the recorded selections."""
    M = _mat(A)
    tau = np.ascontiguousarray(tau, dtype=np.int32)
    Isets = np.ascontiguousarray(Isets, dtype=np.int32).reshape(-1)
    g = _f64(grad_x).copy()
    gb = np.zeros(M.m)
    rc = lib().orc_backward(M.ptr, block_rows, mu, _p(tau), _p(Isets), iters,
                            int(bool(converged)), _p(g), _p(gb))
    if rc:
        raise OracleError(rc, "backward")
    return gb, g


def initial_solution(A, b):
    """Algorithm 2 (appendix): x0 = (<b, A y> / ||A y||^2) y with y the sum of
    the rows of A.  Returns (x0, coefficient)."""
    M = _mat(A)
    b = _f64(b)
    x0 = np.zeros(M.n)
    al = np.zeros(1)
    rc = lib().orc_initial_solution(M.ptr, _p(b), _p(x0), _p(al))
    if rc:
        raise OracleError(rc, "initial_solution")
    return x0, float(al[0])


def fabgmres(A, block_rows: int, mu: float, b, x0=None, seed: int = 0, tol: float = 1e-8,
             max_outer: int = 20, inner_iters: int = 10, eta: float = 1e-1, W=None,
             want_basis: bool = False) -> dict:
    """Algorithm 3 (appendix) in FP64: flexible AB-GMRES with ROR-BK inner
    iterations.  Returns x, the outer steps taken and the residual estimates;
    with want_basis also Z (n x max_outer) and H ((max_outer+1) x max_outer)."""
    M = _mat(A)
    b = _f64(b)
    x = np.zeros(M.n) if x0 is None else _f64(x0).copy()
    Wa = None if W is None else _f64(W)
    outer = np.zeros(1, dtype=np.int64)
    hist = np.zeros(max_outer)
    Z = np.zeros((max_outer, M.n)) if want_basis else None
    H = np.zeros((max_outer, max_outer + 1)) if want_basis else None
    rc = lib().orc_fabgmres(M.ptr, block_rows, mu, _p(b), _p(x), seed & ((1 << 64) - 1), tol,
                            max_outer, inner_iters, eta, _p(Wa), _p(outer), _p(hist), _p(Z), _p(H))
    if rc:
        raise OracleError(rc, "fabgmres")
    k = int(outer[0])
    out = {"x": x, "outer": k, "res_hist": hist[:k].copy()}
    if want_basis:
        out["Z"] = Z[:k].T.copy()                 # n x k
        out["H"] = H[:k, :k + 1].T.copy()          # (k+1) x k
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(t: int) -> None:
    """Threads of the oracle's parallel loops (timing only; results do not
    depend on it)."""
    lib().orc_set_num_threads(int(t))


__all__ = ["ORC_OK", "ORC_ERR_ARG", "ORC_ERR_OOM", "ORC_ERR_NOT_SPD", "ORC_ERR_NONFINITE",
           "Matrix", "OracleError", "num_blocks", "partition", "cosine_rowsums",
           "proposal", "splitmix64_word", "sample", "sample_many", "cholesky",
           "chol_solve", "block_factor", "apply_block", "residual", "topk", "solve", "backward",
           "initial_solution", "fabgmres", "num_threads", "set_num_threads", "lib"]
