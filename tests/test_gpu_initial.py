"""Algorithm 2 (initial solution) on the GPU against the oracle: x0 and the
coefficient, the remark's properties (RRN(x0) <= 1, x0 in the row space), the
zero row sum, FP32 storage, CSR, the full tall workload, and a solve started
from x0 that matches the oracle's solve from the same x0."""
import numpy as np
import pytest

import oracle as O
from workloads import csr_system, dense_svd_system, make

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2510_02156_amd as P  # noqa: E402
from tests.gpu_util import dev, host, rel  # noqa: E402


@pytest.mark.parametrize("m,n,br", [(1000, 300, 20), (300, 5000, 10), (2000, 200, 20)])
def test_initial_solution_dense_fp64(m, n, br):
    s = dense_svd_system(m, n, 1e3, cfg=40 + m)
    sol = P.Solver(dev(s["A"]), br, 1e-3)
    x0, a = sol.initial_solution(dev(s["b"]))
    rx, ra = O.initial_solution(s["A"], s["b"])
    e = rel(host(x0), rx)
    print(f"m={m} n={n}: x0 rel err {e:.2e}, coefficient {a:.6e} vs {ra:.6e}", flush=True)
    assert e < 1e-12 and a == pytest.approx(ra, rel=1e-12)
    r = s["b"] - s["A"] @ host(x0)
    assert np.linalg.norm(r) <= np.linalg.norm(s["b"])
    # reproducible bit for bit
    x1, _ = sol.initial_solution(dev(s["b"]))
    assert torch.equal(x0, x1)


def test_initial_solution_row_space_wide():
    s = dense_svd_system(200, 3000, 1e2, cfg=9, rowspace=True)
    sol = P.Solver(dev(s["A"]), 10, 1e-4)
    x0, _ = sol.initial_solution(dev(s["b"]))
    xh = host(x0)
    A = s["A"]
    null = xh - A.T @ np.linalg.solve(A @ A.T, A @ xh)
    assert np.linalg.norm(null) <= 1e-10 * np.linalg.norm(xh)


def test_initial_solution_zero_row_sum():
    rng = np.random.default_rng(3)
    B = rng.integers(-9, 10, size=(50, 40)).astype(np.float64)
    A = np.vstack([B, -B])
    sol = P.Solver(dev(A), 10, 1e-2)
    x0, a = sol.initial_solution(dev(rng.standard_normal(100)))
    assert a == 0.0 and not torch.any(x0)


def test_initial_solution_fp32_storage():
    s = dense_svd_system(1500, 400, 1e3, cfg=12)
    A32 = s["A"].astype(np.float32)
    Av = A32.astype(np.float64)
    sol = P.Solver(dev(A32, torch.float32), 30, 1e-3, A64=dev(s["A"]))
    # float vectors: everything on the FP32 values
    x0f, af = sol.initial_solution(dev(s["b"], torch.float32))
    rx, ra = O.initial_solution(Av, s["b"].astype(np.float32).astype(np.float64))
    ef = rel(host(x0f), rx)
    # double vectors: the product on the FP64 master (the row sum stays that of the stored values)
    x0d, ad = sol.initial_solution(dev(s["b"]))
    rd, _ = O.initial_solution(s["A"], s["b"])
    ed = rel(host(x0d), rd)
    print(f"fp32 storage: float x0 {ef:.2e}, double x0 {ed:.2e}", flush=True)
    assert x0f.dtype == torch.float32 and ef < 1e-5
    assert x0d.dtype == torch.float64 and ed < 1e-5


def test_initial_solution_csr():
    s = csr_system(3000, 12, cfg=21)
    sol = P.Solver(None, 128, 1.28e-4, rowptr=dev(s["rowptr"], torch.int64),
                   colidx=dev(s["colidx"], torch.int32), values=dev(s["val"]),
                   shape=(s["m"], s["n"]))
    x0, a = sol.initial_solution(dev(s["b"]))
    rx, ra = O.initial_solution(s, s["b"])
    e = rel(host(x0), rx)
    print(f"csr: x0 rel err {e:.2e}", flush=True)
    assert e < 1e-12 and a == pytest.approx(ra, rel=1e-12)


def test_solve_from_initial_solution():
    s = dense_svd_system(800, 250, 1e3, cfg=77)
    br, lam, iters = 20, 1e-3, 30
    sol = P.Solver(dev(s["A"]), br, lam)
    b = dev(s["b"])
    x0, _ = sol.initial_solution(b)
    rx0, _ = O.initial_solution(s["A"], s["b"])
    x, _ = sol.solve(b, x0.clone(), seed=5, tol=0.0, max_iters=iters)
    ref = O.solve(s["A"], br, lam, s["b"], x0=rx0, seed=5, max_iters=iters)
    e = rel(host(x), ref["x"])
    print(f"solve from x0: rel err {e:.2e}", flush=True)
    assert e < 1e-10


@pytest.mark.timeout(600)
def test_initial_solution_full_tall():
    w = make("tall_100000x2000")
    sol = P.Solver(dev(w["A"]), w["block_rows"], w["lam"])
    x0, a = sol.initial_solution(dev(w["b"]))
    rx, ra = O.initial_solution(w["A"], w["b"])
    e = rel(host(x0), rx)
    _, _, rrn0 = sol.residual(dev(w["b"]), x0)
    print(f"full tall: x0 rel err {e:.2e}, RRN(x0) {rrn0:.4f}", flush=True)
    assert e < 1e-12 and rrn0 <= 1.0
