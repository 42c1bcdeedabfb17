"""Seeded synthetic systems with the shapes and spectra of the ROR-BK workloads.

Every array is drawn on the host in FP64 from ``numpy.random.default_rng([cfg,
stream])`` with fixed stream ids, so the oracle and the GPU library are fed the
identical bytes.  Stream ids: 0 = U, 1 = V, 2 = x_star, 3 = sparse columns,
4 = sparse values, 5 = row scales, 6 = x_t (differentiation target), 7 = the
entries of the i.i.d. random dense matrices.

The paper measures on SuiteSparse matrices, AIR Tools II tomography and dense
random matrices (Section 3); none of those data are available here, so these
synthetic systems stand in for the three regimes it covers: tall dense
least-squares, wide dense (minimum-norm target) and sparse ill-conditioned
square.
"""
from __future__ import annotations

import numpy as np

# Stream ids (second word of the numpy seed sequence).
S_U, S_V, S_XSTAR, S_COLS, S_VALS, S_SCALE, S_XT, S_A = range(8)


def haar(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """rows x cols matrix with orthonormal columns, Haar distributed.

    Q factor of a standard-normal matrix with column signs fixed by
    sign(diag R) (Mezzadri's construction), rows >= cols.
    """
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g, mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    q *= d[None, :]
    return q


def log_spaced(count: int, cond: float) -> np.ndarray:
    """Singular values 1 .. 1/cond, log-spaced (s_1 = 1, s_count = 1/cond)."""
    if count == 1:
        return np.ones(1)
    j = np.arange(count, dtype=np.float64)
    return 10.0 ** (-np.log10(cond) * j / (count - 1))


def dense_svd_system(m: int, n: int, cond: float, cfg: int,
                     rowspace: bool = False) -> dict:
    """A = U diag(s) V^T (U, V Haar), planted x_star, consistent b = A x_star.

    With ``rowspace`` the planted solution is V z (in the row space of A), so
    it is the minimum-norm solution of the consistent system.
    """
    ns = min(m, n)
    s = log_spaced(ns, cond)
    u = haar(np.random.default_rng([cfg, S_U]), m, ns)
    v = haar(np.random.default_rng([cfg, S_V]), n, ns)
    u *= s[None, :]
    a = np.ascontiguousarray(u @ v.T)
    del u
    rx = np.random.default_rng([cfg, S_XSTAR])
    if rowspace:
        xstar = v @ rx.standard_normal(ns)
    else:
        xstar = rx.standard_normal(n)
    b = a @ xstar
    return {"format": "dense", "A": a, "b": b, "xstar": xstar, "m": m, "n": n,
            "s": s}


def dense_random_system(m: int, n: int, cfg: int, dist: str = "randn") -> dict:
    """Dense m x n matrix of i.i.d. entries, the random matrices of the
    paper's dense experiments (Tables 3 and 5): ``randn`` draws N(0, 1),
    ``unif1`` draws 1 + U(0, 1).  Planted x_star ~ N(0, 1), consistent
    b = A x_star.  Drawn in row panels so the FP64 matrix is the only large
    allocation.
    """
    ra = np.random.default_rng([cfg, S_A])
    a = np.empty((m, n))
    step = max(1, (1 << 24) // n)
    for r0 in range(0, m, step):
        r1 = min(m, r0 + step)
        if dist == "randn":
            a[r0:r1] = ra.standard_normal((r1 - r0, n))
        elif dist == "unif1":
            a[r0:r1] = 1.0 + ra.uniform(0.0, 1.0, (r1 - r0, n))
        else:
            raise ValueError(dist)
    xstar = np.random.default_rng([cfg, S_XSTAR]).standard_normal(n)
    b = a @ xstar
    return {"format": "dense", "A": a, "b": b, "xstar": xstar, "m": m, "n": n}


def csr_system(m: int, nnz_off: int, cfg: int, scale_lo: float = -6.0) -> dict:
    """Square sparse m x m CSR: per row ``nnz_off`` distinct uniform columns
    other than the diagonal with N(0,1) values, plus A_ii = 1; every row is then
    scaled by 10**U(scale_lo, 0).  Column indices are sorted within each row.
    """
    rc = np.random.default_rng([cfg, S_COLS])
    cols = rc.integers(0, m - 1, size=(m, nnz_off), dtype=np.int64)
    rows = np.arange(m, dtype=np.int64)[:, None]
    cols = cols + (cols >= rows)          # skip the diagonal
    # redraw rows with a repeated column until all are distinct
    while True:
        srt = np.sort(cols, axis=1)
        bad = np.nonzero((srt[:, 1:] == srt[:, :-1]).any(axis=1))[0]
        if bad.size == 0:
            break
        fresh = rc.integers(0, m - 1, size=(bad.size, nnz_off), dtype=np.int64)
        cols[bad] = fresh + (fresh >= bad[:, None])
    vals = np.random.default_rng([cfg, S_VALS]).standard_normal((m, nnz_off))
    allc = np.concatenate([cols, np.arange(m, dtype=np.int64)[:, None]], axis=1)
    allv = np.concatenate([vals, np.ones((m, 1))], axis=1)
    order = np.argsort(allc, axis=1, kind="stable")
    allc = np.take_along_axis(allc, order, axis=1)
    allv = np.take_along_axis(allv, order, axis=1)
    scale = 10.0 ** np.random.default_rng([cfg, S_SCALE]).uniform(scale_lo, 0.0, m)
    allv *= scale[:, None]
    per = nnz_off + 1
    rowptr = np.arange(0, m * per + 1, per, dtype=np.int64)
    colidx = allc.reshape(-1).astype(np.int32)
    val = np.ascontiguousarray(allv.reshape(-1))
    xstar = np.random.default_rng([cfg, S_XSTAR]).standard_normal(m)
    # b = A x_star, row by row in column order
    b = np.add.reduceat(val * xstar[colidx], rowptr[:-1])
    return {"format": "csr", "rowptr": rowptr, "colidx": colidx, "val": val,
            "b": b, "xstar": xstar, "m": m, "n": m}


def to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (round-to-nearest-even via the FP32 value); uint16 bits."""
    f = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    lsb = (f >> 16) & 1
    rounded = (f + np.uint32(0x7FFF) + lsb) >> 16
    return rounded.astype(np.uint16)


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


# The five workloads: shapes, spectra, block sizes and regularization.
#   lam None -> 1e-6 * (rows per block), the paper's default (Section 2, after
#   Theorem 1; Section 3.1).
WORKLOADS = {
    "dense_2000x200": dict(cfg=1, kind="dense", m=2000, n=200, cond=1e6,
                           block_rows=20, lam=1e-3, tol=1e-8, max_iters=5000),
    "tall_100000x2000": dict(cfg=2, kind="dense", m=100000, n=2000, cond=1e8,
                             block_rows=64, lam=1e-4, tol=1e-8, max_iters=5000),
    "csr_200000": dict(cfg=3, kind="csr", m=200000, nnz_off=12,
                       block_rows=128, lam=None, tol=1e-8, max_iters=5000),
    "wide_2000x50000": dict(cfg=4, kind="dense", m=2000, n=50000, cond=1e6,
                            rowspace=True, block_rows=32, lam=1e-4, tol=1e-8,
                            max_iters=5000),
    "diff_20000x1000": dict(cfg=5, kind="dense", m=20000, n=1000, cond=1e5,
                            f32=True, block_rows=50, lam=None, tol=0.0,
                            max_iters=300, checkpoint_every=20),
    # the paper's own protocol (Section 3.1): 100 blocks, lambda = 1e-6 * rows
    # per block, stop at RRN < 1e-6; shapes of Table 3 (randn) and Table 5
    # (1 + U(0,1))
    "randn_60000x10000": dict(cfg=6, kind="randn", m=60000, n=10000,
                              block_rows=600, lam=None, tol=1e-6, max_iters=2000),
    "unif_100000x10000": dict(cfg=7, kind="unif1", m=100000, n=10000,
                              block_rows=1000, lam=None, tol=1e-6, max_iters=2000),
    "unif_100000x15000": dict(cfg=10, kind="unif1", m=100000, n=15000,
                              block_rows=1000, lam=None, tol=1e-6, max_iters=2000),
    "unif_100000x20000": dict(cfg=9, kind="unif1", m=100000, n=20000,
                              block_rows=1000, lam=None, tol=1e-6, max_iters=2000),
    # supplementary system for time to 1e-8: the tall workload's shape, blocks,
    # regularisation and generator at a low condition number, where plain
    # ROR-BK reaches a relative residual of 1e-8 within the 5000-iteration
    # cap (at cond 1e8 it levels off near 5e-3)
    "tall_cond10_100000x2000": dict(cfg=11, kind="dense", m=100000, n=2000, cond=10.0,
                                    block_rows=64, lam=1e-4, tol=1e-8, max_iters=5000),
    # tall and narrow with the paper's 100 blocks: blocks of 2000 rows against
    # 500 columns, the case for the column form of the block solve (Sec. 3.1)
    "colform_200000x500": dict(cfg=8, kind="dense", m=200000, n=500, cond=1e6,
                               block_rows=2000, lam=None, tol=1e-8, max_iters=2000),
}


def make(name: str, m: int | None = None, n: int | None = None) -> dict:
    """Build workload ``name``; ``m``/``n`` override the sizes (same recipe)."""
    w = dict(WORKLOADS[name])
    cfg = w["cfg"]
    if w["kind"] == "csr":
        mm = m or w["m"]
        sysd = csr_system(mm, w["nnz_off"], cfg)
    elif w["kind"] in ("randn", "unif1"):
        sysd = dense_random_system(m or w["m"], n or w["n"], cfg, w["kind"])
    else:
        mm, nn = m or w["m"], n or w["n"]
        sysd = dense_svd_system(mm, nn, w["cond"], cfg,
                                rowspace=w.get("rowspace", False))
        if w.get("f32"):
            a32 = sysd["A"].astype(np.float32)
            sysd["A"] = a32.astype(np.float64)      # FP64 view of the FP32 values
            sysd["A32"] = a32
            sysd["b"] = sysd["A"] @ sysd["xstar"]
            sysd["xt"] = np.random.default_rng([cfg, S_XT]).standard_normal(nn)
    lam = w["lam"] if w["lam"] is not None else 1e-6 * w["block_rows"]
    sysd.update(name=name, block_rows=w["block_rows"], lam=lam, tol=w["tol"],
                max_iters=w["max_iters"], seed=1000 * cfg + 7,
                checkpoint_every=w.get("checkpoint_every", 0))
    return sysd
