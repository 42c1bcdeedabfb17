"""FP32 / BF16 storage paths and FP64 iterative refinement against the oracle.

FP32 and BF16 solves are compared with the FP64 oracle run on the same stored
values (the FP32- or BF16-rounded matrix, upcast), replaying the oracle's
selections.  Tolerance: the passes accumulate in FP32 (unit roundoff 6e-8) over
a few thousand terms per product and tens of contractive block steps, so 1e-4
relative on x is the derived bar (measured errors are printed).
"""
import numpy as np
import pytest

import oracle as O
from workloads import dense_svd_system

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2510_02156_amd as P  # noqa: E402
from tests.gpu_util import bf16_tensor, bf16_values, dev, host, rel  # noqa: E402

TOL_F32 = 1e-4

CASES = [(1000, 300, 20, 1e-3, 1e3), (600, 2500, 32, 1e-4, 1e3), (900, 130, 64, 1e-3, 1e2)]


@pytest.mark.parametrize("m,n,br,lam,cond", CASES)
@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_low_precision_replay(m, n, br, lam, cond, storage):
    s = dense_svd_system(m, n, cond, cfg=300 + m)
    if storage == "f32":
        Av = s["A"].astype(np.float32).astype(np.float64)
        At = dev(s["A"], torch.float32)
    else:
        Av = bf16_values(s["A"])
        At = bf16_tensor(s["A"])
    b = Av @ s["xstar"]
    iters = 40
    ref = O.solve(Av, br, lam, b, seed=4, max_iters=iters)
    sol = P.Solver(At, br, lam)
    sol.set_replay(ref["tau"], ref["I"], iters)
    x, info = sol.solve(dev(b, torch.float32), seed=0, tol=0.0, max_iters=iters, replay=True)
    e = rel(host(x), ref["x"])
    print(f"{storage} m={m} n={n}: rel err vs FP64 oracle {e:.2e}", flush=True)
    assert x.dtype == torch.float32
    assert e < TOL_F32


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_low_precision_setup(storage):
    s = dense_svd_system(800, 200, 1e3, cfg=77)
    Av = s["A"].astype(np.float32).astype(np.float64) if storage == "f32" else bf16_values(s["A"])
    At = dev(s["A"], torch.float32) if storage == "f32" else bf16_tensor(s["A"])
    sol = P.Solver(At, 20, 1e-3)
    got = sol.setup_arrays()
    S = O.cosine_rowsums(Av, 20)
    np.testing.assert_allclose(got["S"], S, rtol=1e-12)   # setup runs in FP64 on the stored values
    off = O.partition(800, 20)
    for t in (0, 17, 39):
        L = O.block_factor(Av, np.arange(off[t], off[t + 1]), 1e-3)
        Hinv = np.linalg.inv(L @ L.T)
        assert rel(sol.block_inverse(t), Hinv) < 1e-10


def test_refine_fp64_inner_is_restart_equivalent():
    """FP64 refinement (FP64 inner solve) reproduces the plain FP64 trajectory
    up to rounding: block Kaczmarz restarted on (A, b - A x, 0) equals
    continuing on (A, b, x) with the same selections."""
    s = dense_svd_system(1200, 150, 10.0, cfg=21)
    A = dev(s["A"])
    b = dev(s["b"])
    sol = P.Solver(A, 24, 1e-4, A64=A)
    sol.set_refine(10, 0.0)
    x1, i1 = sol.solve(b, seed=8, tol=0.0, max_iters=60)
    x2, i2 = sol.solve(b, seed=8, tol=0.0, max_iters=60, refine=True)
    assert i2["n_refine"] == 6 and i2["iters"] == 60
    e = rel(host(x2), host(x1))
    print(f"refine(FP64 inner) vs plain: {e:.2e}", flush=True)
    assert e < 1e-9


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_refine_reaches_tolerance(storage):
    """Well-conditioned system: FP32/BF16 passes + FP64 refinement reach
    ||b - A x|| / ||b|| < 1e-8 (beyond what FP32 arithmetic alone resolves)."""
    s = dense_svd_system(3000, 200, 10.0, cfg=31)
    A64 = dev(s["A"])
    At = A64.float() if storage == "f32" else bf16_tensor(s["A"])
    b = dev(s["b"])
    sol = P.Solver(At, 30, 1e-6, A64=A64)
    sol.set_refine(40, 1e-4)
    x, info = sol.solve(b, seed=3, tol=1e-8, max_iters=4000, refine=True)
    print(f"{storage}+refine: iters {info['iters']} rrn {info['rrn']:.2e} steps {info['n_refine']}", flush=True)
    assert info["converged"] and info["rrn"] < 1e-8
    r = s["b"] - s["A"] @ host(x)
    assert np.linalg.norm(r) / np.linalg.norm(s["b"]) < 1e-8
    assert rel(host(x), s["xstar"]) < 1e-6
    ref = O.solve(s["A"], 30, 1e-6, s["b"], seed=3, tol=1e-8, max_iters=4000, record=False)
    assert ref["converged"]
    print(f"oracle FP64: iters {ref['iters']}; rel diff of solutions {rel(host(x), ref['x']):.2e}")
    assert rel(host(x), ref["x"]) < 1e-6


def test_refine_requires_master():
    s = dense_svd_system(200, 30, 10.0, cfg=5)
    sol = P.Solver(dev(s["A"], torch.float32), 10, 1e-3)
    with pytest.raises(P.RorBkError) as e:
        sol.solve(dev(s["b"]), seed=1, tol=1e-8, max_iters=10, refine=True)
    assert e.value.code == P.RORBK_ERR_INVALID_ARG


# BF16 rows whose stride is 4 mod 8 elements (rows start 16-byte aligned or
# half a vector past it, alternately): the residual pass reads them with
# aligned loads moved back by half a vector; the last row's end takes the
# element-wise path.  Strides 0 mod 8 and 2 mod 8 take the other two forms.
@pytest.mark.parametrize("m,n,br", [(1, 500, 1), (3, 12, 2), (7, 500, 3), (130, 300, 16),
                                    (40, 1020, 8), (129, 2500, 32), (65, 4100, 16),
                                    (33, 130, 8), (17, 512, 4)])
def test_bf16_residual_row_strides(m, n, br):
    rng = np.random.default_rng(m * 7919 + n)
    A = rng.standard_normal((m, n))
    Av = bf16_values(A)
    x = rng.standard_normal(n).astype(np.float32).astype(np.float64)
    b = rng.standard_normal(m).astype(np.float32).astype(np.float64)
    sol = P.Solver(bf16_tensor(A), br, 1e-3)
    r, _, _ = sol.residual(dev(b, torch.float32), dev(x, torch.float32))
    rr = b - Av @ x
    scale = np.abs(Av) @ np.abs(x) + np.abs(b)
    # FP32 products summed in FP32 (each lane in column order, then a six-level
    # butterfly), then r rounded to FP32: at most n + 8 roundings per term
    bound = (n + 8) * 2.0 ** -24 * scale * 1.01
    err = np.abs(host(r) - rr)
    print(f"bf16 residual m={m} n={n}: max err / bound {np.max(err / bound):.3f}", flush=True)
    assert np.all(err <= bound)
