"""Algorithm 3 (flexible AB-GMRES with ROR-BK inner iterations) on the GPU
against the FP64 oracle: the same inner draws and greedy sets, so the outer
step count, the result and its residual agree; the row-space remark; CSR;
convergence to the tolerance; argument checks."""
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


@pytest.mark.parametrize("m,n,br,outer,inner", [(300, 120, 20, 10, 3), (500, 60, 25, 8, 5),
                                                (150, 700, 15, 6, 4)])
def test_fabgmres_matches_oracle(m, n, br, outer, inner):
    s = dense_svd_system(m, n, 1e3, cfg=70 + m)
    lam, eta = 1e-3, 1e-2
    ref = O.fabgmres(s["A"], br, lam, s["b"], seed=6, tol=1e-12, max_outer=outer,
                     inner_iters=inner, eta=eta)
    sol = P.Solver(dev(s["A"]), br, lam)
    x, info = sol.fabgmres(dev(s["b"]), seed=6, tol=1e-12, max_outer=outer, inner_iters=inner,
                           eta=eta)
    e = rel(host(x), ref["x"])
    rr = np.linalg.norm(s["b"] - s["A"] @ ref["x"]) / np.linalg.norm(s["b"])
    print(f"m={m} n={n}: outer {info['outer']} vs {ref['outer']}, x rel err {e:.2e}, "
          f"rrn {info['rrn']:.3e} vs {rr:.3e}", flush=True)
    assert info["outer"] == ref["outer"]
    assert e < 1e-9
    assert info["rrn"] == pytest.approx(rr, rel=1e-7)
    assert info["rrn"] == pytest.approx(ref["res_hist"][-1], rel=1e-6)


def test_fabgmres_row_space_and_initial_point():
    s = dense_svd_system(80, 400, 1e2, cfg=71, rowspace=True)
    A = s["A"]
    sol = P.Solver(dev(A), 10, 1e-4)
    b = dev(s["b"])
    x0, _ = sol.initial_solution(b)                       # Algorithm 2: in R(A^T)
    x, info = sol.fabgmres(b, x0.clone(), seed=1, tol=1e-10, max_outer=8, inner_iters=2, eta=1e-6)
    xh = host(x)
    null = xh - A.T @ np.linalg.solve(A @ A.T, A @ xh)
    assert np.linalg.norm(null) <= 1e-9 * np.linalg.norm(xh)
    ref = O.fabgmres(A, 10, 1e-4, s["b"], x0=O.initial_solution(A, s["b"])[0], seed=1, tol=1e-10,
                     max_outer=8, inner_iters=2, eta=1e-6)
    assert rel(xh, ref["x"]) < 1e-9


def test_fabgmres_csr():
    s = csr_system(2000, 12, cfg=72)
    br, lam = 64, 1e-4
    ref = O.fabgmres(s, br, lam, s["b"], seed=3, tol=1e-12, max_outer=6, inner_iters=3, eta=1e-3)
    sol = P.Solver(None, br, lam, rowptr=dev(s["rowptr"], torch.int64),
                   colidx=dev(s["colidx"], torch.int32), values=dev(s["val"]),
                   shape=(s["m"], s["n"]))
    x, info = sol.fabgmres(dev(s["b"]), seed=3, tol=1e-12, max_outer=6, inner_iters=3, eta=1e-3)
    e = rel(host(x), ref["x"])
    print(f"csr: outer {info['outer']}, x rel err {e:.2e}", flush=True)
    assert info["outer"] == ref["outer"] and e < 1e-9


def test_fabgmres_reaches_tolerance():
    s = dense_svd_system(400, 100, 10.0, cfg=73)
    sol = P.Solver(dev(s["A"]), 20, 1e-6)
    x, info = sol.fabgmres(dev(s["b"]), seed=2, tol=1e-10, max_outer=40, inner_iters=5, eta=1e-2)
    r = s["b"] - s["A"] @ host(x)
    print(f"converged {info['converged']} after {info['outer']} outer / {info['inner_iters']} "
          f"inner iterations, rrn {info['rrn']:.2e}", flush=True)
    assert info["converged"] and info["rrn"] < 1e-9
    assert np.linalg.norm(r) / np.linalg.norm(s["b"]) < 1e-9


def test_fabgmres_arguments():
    s = dense_svd_system(100, 30, 10.0, cfg=74)
    sol = P.Solver(dev(s["A"]), 10, 1e-3)
    with pytest.raises(P.RorBkError):
        sol.fabgmres(dev(s["b"]), max_outer=0)
    s32 = P.Solver(dev(s["A"], torch.float32), 10, 1e-3)
    with pytest.raises(P.RorBkError) as e:
        s32.fabgmres(dev(s["b"]))
    assert e.value.code == P.RORBK_ERR_UNSUPPORTED
