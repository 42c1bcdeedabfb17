"""Adjoint (reverse-mode) parity: GPU backward vs the FP64 oracle's adjoint on
the same recorded selections, record vs checkpoint recomputation (bit
identical), exact central differences with replayed selections, the autograd
wrapper, and the FP32 adjoint against the FP64 reference.
"""
import numpy as np
import pytest

import oracle as O
from workloads import dense_svd_system, make

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2510_02156_amd as P  # noqa: E402
from tests.gpu_util import dev, host, rel  # noqa: E402


def setup_case(m=600, n=120, br=20, lam=1e-3, cond=1e3, cfg=51):
    s = dense_svd_system(m, n, cond, cfg=cfg)
    rng = np.random.default_rng(cfg)
    s["x0"] = rng.standard_normal(n)
    s["xt"] = rng.standard_normal(n)
    return s, br, lam


@pytest.mark.parametrize("m,n,br", [(600, 120, 20), (400, 900, 16), (500, 64, 65)])
def test_backward_matches_oracle(m, n, br):
    s, _, lam = setup_case(m, n, br)
    iters = 25
    sol = P.Solver(dev(s["A"]), br, lam)
    x, info = sol.solve(dev(s["b"]), dev(s["x0"]), seed=9, tol=0.0, max_iters=iters, record=True)
    rec = sol.record()
    g = 2 * (host(x) - s["xt"])
    gb, gx0 = sol.backward(dev(g))
    rb, rx0 = O.backward(s["A"], br, lam, rec["tau"], rec["I"], iters, False, g)
    eb, ex = rel(host(gb), rb), rel(host(gx0), rx0)
    print(f"m={m} n={n} br={br}: dL/db {eb:.2e}, dL/dx0 {ex:.2e}", flush=True)
    assert eb < 1e-10 and ex < 1e-10


def test_checkpoint_equals_record_bitwise():
    s, br, lam = setup_case()
    iters = 37
    sol = P.Solver(dev(s["A"]), br, lam)
    b = dev(s["b"])
    x1, _ = sol.solve(b, dev(s["x0"]), seed=2, tol=0.0, max_iters=iters, record=True)
    g = dev(2 * (host(x1) - s["xt"]))
    gb1, gx1 = sol.backward(g)
    x2, _ = sol.solve(b, dev(s["x0"]), seed=2, tol=0.0, max_iters=iters, checkpoint_every=8)
    assert torch.equal(x1, x2)
    gb2, gx2 = sol.backward(g)
    assert torch.equal(gb1, gb2) and torch.equal(gx1, gx2)


def test_backward_converged_run():
    s, br, lam = setup_case(cond=10.0)
    sol = P.Solver(dev(s["A"]), br, lam)
    x, info = sol.solve(dev(s["b"]), dev(s["x0"]), seed=5, tol=0.3, max_iters=100, record=True)
    assert info["converged"]
    rec = sol.record()
    g = 2 * (host(x) - s["xt"])
    gb, gx0 = sol.backward(dev(g))
    rb, rx0 = O.backward(s["A"], br, lam, rec["tau"], rec["I"], info["iters"], True, g)
    assert rel(host(gb), rb) < 1e-10 and rel(host(gx0), rx0) < 1e-10
    # checkpointed recomputation stops at the same iteration
    sol.solve(dev(s["b"]), dev(s["x0"]), seed=5, tol=0.3, max_iters=100, checkpoint_every=3)
    gb2, gx2 = sol.backward(dev(g))
    assert torch.equal(gb, gb2) and torch.equal(gx0, gx2)


def test_finite_differences_exact():
    """With the selections replayed, x_K is linear in (b, x0) and
    L = ||x_K - x_t||^2 quadratic: central differences are exact up to
    rounding."""
    s, br, lam = setup_case(m=300, n=60, br=15)
    iters = 12
    sol = P.Solver(dev(s["A"]), br, lam)
    x, _ = sol.solve(dev(s["b"]), dev(s["x0"]), seed=4, tol=0.0, max_iters=iters, record=True)
    rec = sol.record()
    g = 2 * (host(x) - s["xt"])
    gb, gx0 = sol.backward(dev(g))
    sol.set_replay(rec["tau"], rec["I"], iters)

    def loss(bv, x0v):
        xx, _ = sol.solve(dev(bv), dev(x0v), seed=0, tol=0.0, max_iters=iters, replay=True)
        return float(np.sum((host(xx) - s["xt"]) ** 2))

    h = 1e-3
    for i in (0, 77, 299):
        e = np.zeros(300); e[i] = h
        fd = (loss(s["b"] + e, s["x0"]) - loss(s["b"] - e, s["x0"])) / (2 * h)
        assert fd == pytest.approx(float(host(gb)[i]), rel=1e-6, abs=1e-9)
    for i in (0, 59):
        e = np.zeros(60); e[i] = h
        fd = (loss(s["b"], s["x0"] + e) - loss(s["b"], s["x0"] - e)) / (2 * h)
        assert fd == pytest.approx(float(host(gx0)[i]), rel=1e-6, abs=1e-9)


def test_autograd_function():
    s, br, lam = setup_case()
    sol = P.Solver(dev(s["A"]), br, lam)
    b = dev(s["b"]).requires_grad_(True)
    x0 = dev(s["x0"]).requires_grad_(True)
    xt = dev(s["xt"])
    xk = P.RorBkFunction.apply(b, x0, sol, 6, 20, 0)
    loss = ((xk - xt) ** 2).sum()
    loss.backward()
    rec = sol.record()
    g = 2 * (host(xk.detach()) - s["xt"])
    rb, rx0 = O.backward(s["A"], br, lam, rec["tau"], rec["I"], 20, False, g)
    assert rel(host(b.grad), rb) < 1e-10 and rel(host(x0.grad), rx0) < 1e-10
    # checkpointed variant gives the same gradients
    b2 = dev(s["b"]).requires_grad_(True)
    x02 = dev(s["x0"]).requires_grad_(True)
    xk2 = P.RorBkFunction.apply(b2, x02, sol, 6, 20, 5)
    ((xk2 - xt) ** 2).sum().backward()
    assert torch.equal(b.grad, b2.grad) and torch.equal(x0.grad, x02.grad)


def test_fp32_adjoint_vs_fp64_reference():
    """FP32 storage and vectors; reference: the FP64 oracle adjoint on the
    FP32 values upcast, same recorded selections.  Bar 1e-4 (FP32 passes)."""
    s = dense_svd_system(2000, 200, 1e3, cfg=61)
    A32 = s["A"].astype(np.float32)
    Av = A32.astype(np.float64)
    b = Av @ s["xstar"]
    xt = np.random.default_rng(1).standard_normal(200)
    sol = P.Solver(dev(A32, torch.float32), 50, 5e-5)
    iters = 30
    x, _ = sol.solve(dev(b, torch.float32), seed=7, tol=0.0, max_iters=iters, record=True)
    rec = sol.record()
    g = 2 * (host(x).astype(np.float64) - xt)
    gb, gx0 = sol.backward(dev(g, torch.float32))
    rb, rx0 = O.backward(Av, 50, 5e-5, rec["tau"], rec["I"], iters, False, g)
    eb, ex = rel(host(gb), rb), rel(host(gx0), rx0)
    print(f"FP32 adjoint vs FP64: dL/db {eb:.2e}, dL/dx0 {ex:.2e}", flush=True)
    assert eb < 1e-4 and ex < 1e-4


def test_differentiation_workload_full_size():
    """The differentiation workload at full size: A 20000 x 1000 FP32 (cond
    1e5), blocks of 50, K = 300 iterations, checkpoints every 20, loss
    ||x_K - x_t||^2.  The FP32 adjoint is checked against the FP64 oracle
    adjoint on the same selections, and against central differences of the FP64
    forward (replayed selections) on sampled coordinates of b."""
    w = make("diff_20000x1000")
    A32 = w["A32"]
    Av = w["A"]
    b = w["b"]
    sol = P.Solver(dev(A32, torch.float32), w["block_rows"], w["lam"])
    iters, c = w["max_iters"], w["checkpoint_every"]
    x, info = sol.solve(dev(b, torch.float32), seed=w["seed"], tol=0.0, max_iters=iters,
                        checkpoint_every=c)
    assert info["iters"] == iters
    g = 2 * (host(x).astype(np.float64) - w["xt"])
    gb, gx0 = sol.backward(dev(g, torch.float32))
    rec = sol.record()
    rb, rx0 = O.backward(Av, w["block_rows"], w["lam"], rec["tau"], rec["I"], iters, False, g)
    eb, ex = rel(host(gb), rb), rel(host(gx0), rx0)
    print(f"full-size FP32 adjoint vs FP64: dL/db {eb:.2e}, dL/dx0 {ex:.2e}", flush=True)
    assert eb < 1e-3 and ex < 1e-3
    # central differences of the FP64 forward with replayed selections
    s64 = P.Solver(dev(Av), w["block_rows"], w["lam"])
    s64.set_replay(rec["tau"], rec["I"], iters)
    x64, _ = s64.solve(dev(b), seed=0, tol=0.0, max_iters=iters, replay=True)
    g64 = 2 * (host(x64) - w["xt"])
    s64.solve(dev(b), seed=0, tol=0.0, max_iters=iters, replay=True, record=True)
    gb64, _ = s64.backward(dev(g64))

    def loss(bv):
        xx, _ = s64.solve(dev(bv), seed=0, tol=0.0, max_iters=iters, replay=True)
        return float(np.sum((host(xx) - w["xt"]) ** 2))

    h = 1e-2
    for i in (0, 12345, 19999):
        e = np.zeros(len(b)); e[i] = h
        fd = (loss(b + e) - loss(b - e)) / (2 * h)
        assert fd == pytest.approx(float(host(gb64)[i]), rel=1e-5, abs=1e-8)


def test_autograd_interleaved_forwards_are_refused():
    """Two differentiated forwards on one Solver before their backwards: the
    second replaced the handle's record, so the first graph's backward raises
    instead of returning the second run's gradients; with one Solver per
    forward both backwards match the oracle's adjoint of their own run."""
    s, br, lam = setup_case()
    iters = 12
    sol = P.Solver(dev(s["A"]), br, lam)
    b1 = dev(s["b"]).requires_grad_(True)
    b2 = dev(2.0 * s["b"]).requires_grad_(True)
    x0 = dev(s["x0"])
    xa = P.RorBkFunction.apply(b1, x0, sol, 3, iters, 0)
    xb = P.RorBkFunction.apply(b2, x0, sol, 4, iters, 0)
    xt = dev(s["xt"])
    with pytest.raises(RuntimeError, match="another solve"):
        ((xa - xt) ** 2).sum().backward()
    ((xb - xt) ** 2).sum().backward()        # the latest forward still differentiates
    assert b2.grad is not None
    # separate solvers: each graph keeps its own record
    s1, s2 = P.Solver(dev(s["A"]), br, lam), P.Solver(dev(s["A"]), br, lam)
    c1 = dev(s["b"]).requires_grad_(True)
    c2 = dev(2.0 * s["b"]).requires_grad_(True)
    ya = P.RorBkFunction.apply(c1, x0, s1, 3, iters, 0)
    yb = P.RorBkFunction.apply(c2, x0, s2, 4, iters, 0)
    for y, c, so in ((ya, c1, s1), (yb, c2, s2)):
        ((y - xt) ** 2).sum().backward()
        rec = so.record()
        g = 2 * (host(y.detach()) - s["xt"])
        rb, _ = O.backward(s["A"], br, lam, rec["tau"], rec["I"], iters, False, g)
        assert rel(host(c.grad), rb) < 1e-10
