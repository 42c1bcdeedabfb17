"""Degenerate shapes and inputs on the GPU against the oracle: blocks of one
row (Kaczmarz projections and Motzkin's greedy row), one block of all rows,
a single column, CSR rows without entries, and the error paths for them."""
import numpy as np
import pytest

import oracle as O
from workloads import csr_system, dense_svd_system

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2510_02156_amd as P  # noqa: E402
from tests.gpu_util import dev, host, rel  # noqa: E402


def run_both(A, br, lam, b, iters=30, seed=3, csr=None):
    ref = O.solve(csr if csr is not None else A, br, lam, b, seed=seed, max_iters=iters)
    if csr is not None:
        sol = P.Solver(None, br, lam, rowptr=dev(csr["rowptr"], torch.int64),
                       colidx=dev(csr["colidx"], torch.int32), values=dev(csr["val"]),
                       shape=(csr["m"], csr["n"]))
    else:
        sol = P.Solver(dev(A), br, lam)
    x, info = sol.solve(dev(b), seed=seed, tol=0.0, max_iters=iters, record=True)
    rec = sol.record()
    np.testing.assert_array_equal(rec["tau"], ref["tau"])
    np.testing.assert_array_equal(rec["I"], ref["I"])
    return host(x), ref["x"], sol


def test_blocks_of_one_row_kaczmarz():
    """block_rows = 1 and lambda = 0: every step is a Kaczmarz projection (the
    row's residual vanishes) and the greedy row is Motzkin's."""
    s = dense_svd_system(60, 25, 10.0, cfg=1)
    x, rx, sol = run_both(s["A"], 1, 0.0, s["b"])
    assert sol.k == 60 and sol.K == 1
    assert rel(x, rx) < 1e-10
    # one more sampled step from x: the sampled row's residual is zero after it
    r_prev = s["b"] - s["A"] @ x
    i = int(np.argmax(np.abs(r_prev)))
    x1 = O.apply_block(s["A"], [i], 0.0, s["b"], x)
    assert abs(s["b"][i] - s["A"][i] @ x1) <= 1e-12 * np.linalg.norm(s["A"][i]) * np.linalg.norm(x1)


def test_one_block_of_all_rows():
    """block_rows = m: one block, and the greedy set is every row."""
    s = dense_svd_system(120, 300, 1e2, cfg=2)
    x, rx, sol = run_both(s["A"], 120, 1e-3, s["b"], iters=5)
    assert sol.k == 1 and sol.K == 120
    assert rel(x, rx) < 1e-10


def test_single_column():
    s = dense_svd_system(100, 1, 1.0, cfg=3)
    x, rx, _ = run_both(s["A"], 10, 1e-3, s["b"])
    assert rel(x, rx) < 1e-12


def test_csr_rows_without_entries():
    s = csr_system(600, 4, cfg=4)
    rp, ci, va = s["rowptr"], s["colidx"], s["val"]
    keep = np.ones(600, dtype=bool)
    keep[[5, 6, 7, 300, 599]] = False              # these rows lose every entry
    lens = np.diff(rp) * keep
    rows = np.repeat(np.arange(600), np.diff(rp))
    mask = keep[rows]
    csr = {"format": "csr", "m": 600, "n": 600, "rowptr": np.concatenate([[0], np.cumsum(lens)]),
           "colidx": ci[mask], "val": va[mask]}
    b = O.residual(csr, np.zeros(600), -s["xstar"])
    x, rx, _ = run_both(None, 20, 1e-3, b, csr=csr)
    assert rel(x, rx) < 1e-10
    with pytest.raises(P.RorBkError) as e:     # lambda = 0: the empty rows make a block singular
        P.Solver(None, 20, 0.0, rowptr=dev(csr["rowptr"], torch.int64),
                 colidx=dev(csr["colidx"], torch.int32), values=dev(csr["val"]),
                 shape=(600, 600))
    assert e.value.code == P.RORBK_ERR_NOT_SPD


def test_replay_arguments_checked():
    s = dense_svd_system(100, 30, 10.0, cfg=5)
    sol = P.Solver(dev(s["A"]), 10, 1e-3)
    tau = np.zeros(3, dtype=np.int32)
    with pytest.raises(P.RorBkError):
        sol.set_replay(tau, np.array([5, 3] + [0] * 8, dtype=np.int32), 1)   # not ascending
    with pytest.raises(P.RorBkError):
        sol.set_replay(np.array([0, 10, 0], dtype=np.int32), np.arange(10, dtype=np.int32), 1)
