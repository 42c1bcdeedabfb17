"""GPU parity of the CSR path against the FP64 oracle (the sparse square
workload: rows of 12 random off-diagonal N(0,1) entries plus a unit diagonal,
rows scaled by 10^U(-6,0)).

Bars as for the dense path: integer results (draws, greedy sets) bit-exact,
FP64 vectors and stored inverses within the stated relative tolerances, FP32
values within 1e-4 of the oracle run on the same rounded values with its
selections replayed.
"""
import numpy as np
import pytest

import oracle as O
from workloads import csr_system, make

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2510_02156_amd as P  # noqa: E402
from tests.gpu_util import dev, host, rel  # noqa: E402

# m, nnz per row (off-diagonal), block rows, lambda   (ragged partitions)
# the last case has more block entries than one update chunk or the next-row
# prefetch holds (31 per row x 100 rows)
CASES = [(3000, 12, 128, 1.28e-4), (2011, 12, 64, 1e-4), (1500, 5, 33, 1e-3), (900, 12, 129, 1e-3),
         (1000, 30, 100, 1e-3)]


def system(m, nnz_off, cfg=7, scale_lo=-6.0):
    return csr_system(m, nnz_off, cfg=cfg + m, scale_lo=scale_lo)


def solver(s, br, lam, values=None, A64=None):
    vals = dev(s["val"]) if values is None else values
    return P.Solver(None, br, lam, rowptr=dev(s["rowptr"], torch.int64),
                    colidx=dev(s["colidx"], torch.int32), values=vals,
                    shape=(s["m"], s["n"]), A64=A64)


@pytest.mark.parametrize("m,nz,br,lam", CASES)
def test_csr_setup_matches_oracle(m, nz, br, lam):
    s = system(m, nz)
    print(f"csr setup m={m} br={br}", flush=True)
    sol = solver(s, br, lam)
    got = sol.setup_arrays()
    np.testing.assert_array_equal(got["offsets"], O.partition(m, br))
    S = O.cosine_rowsums(s, br)
    np.testing.assert_allclose(got["S"], S, rtol=1e-12)
    Pbar, W = O.proposal(S, s["n"])
    np.testing.assert_allclose(got["pbar"], Pbar, rtol=1e-12)
    np.testing.assert_allclose(got["W"], W, rtol=1e-12)
    off = got["offsets"]
    for t in sorted({0, sol.k // 2, sol.k - 1}):
        rows = np.arange(off[t], off[t + 1])
        L = O.block_factor(s, rows, lam)
        Hinv = np.linalg.inv(L @ L.T)
        assert rel(sol.block_inverse(t), Hinv) < 50 * np.linalg.cond(L @ L.T) * np.finfo(float).eps


@pytest.mark.parametrize("m,nz,br,lam", CASES[:2])
def test_csr_residual_and_block_norms(m, nz, br, lam):
    s = system(m, nz)
    x = np.random.default_rng(5).standard_normal(m)
    sol = solver(s, br, lam)
    r, bn, rrn = sol.residual(dev(s["b"]), dev(x))
    rr = O.residual(s, s["b"], x)
    assert rel(host(r), rr) < 1e-13
    off = O.partition(m, br)
    bref = np.array([np.sum(rr[off[t]:off[t + 1]] ** 2) for t in range(len(off) - 1)])
    np.testing.assert_allclose(host(bn), bref, rtol=1e-12)
    assert abs(rrn - np.linalg.norm(rr) / np.linalg.norm(s["b"])) < 1e-13 * max(rrn, 1e-300)


@pytest.mark.parametrize("m,nz,br,lam", CASES)
def test_csr_replay_trajectory_fp64(m, nz, br, lam):
    s = system(m, nz)
    iters = 40
    ref = O.solve(s, br, lam, s["b"], seed=3, max_iters=iters)
    sol = solver(s, br, lam)
    sol.set_replay(ref["tau"], ref["I"], iters)
    x, info = sol.solve(dev(s["b"]), seed=0, tol=0.0, max_iters=iters, replay=True)
    e = rel(host(x), ref["x"])
    print(f"csr m={m} br={br}: replay rel err {e:.2e}", flush=True)
    assert info["iters"] == iters
    assert e < 1e-10


@pytest.mark.parametrize("m,nz,br,lam", CASES[:3])
def test_csr_free_running_matches_oracle(m, nz, br, lam):
    s = system(m, nz)
    iters = 30
    ref = O.solve(s, br, lam, s["b"], seed=11, max_iters=iters)
    sol = solver(s, br, lam)
    x, info = sol.solve(dev(s["b"]), seed=11, tol=0.0, max_iters=iters, record=True)
    rec = sol.record()
    np.testing.assert_array_equal(rec["tau"], ref["tau"])
    np.testing.assert_array_equal(rec["I"], ref["I"])
    e = rel(host(x), ref["x"])
    print(f"csr m={m}: free-running rel err {e:.2e}", flush=True)
    assert e < 1e-10
    np.testing.assert_allclose(rec["rrn"], ref["rrn_hist"], rtol=1e-9)


def test_csr_stop_test_and_resume():
    s = system(2000, 12, scale_lo=0.0)
    br, lam = 50, 1e-4
    ref = O.solve(s, br, lam, s["b"], seed=4, tol=0.5, max_iters=200)
    sol = solver(s, br, lam)
    x, info = sol.solve(dev(s["b"]), seed=4, tol=0.5, max_iters=200)
    assert info["iters"] == ref["iters"] and info["converged"] == ref["converged"]
    # resume: 10 iterations, then 15 more from start_iter 10, equals 25 at once
    b = dev(s["b"])
    x1, _ = sol.solve(b, seed=8, tol=0.0, max_iters=25)
    x2, _ = sol.solve(b, seed=8, tol=0.0, max_iters=10)
    x2, _ = sol.solve(b, x2, seed=8, tol=0.0, max_iters=15, start_iter=10)
    assert torch.equal(x1, x2)


def test_csr_fp32_values_replay():
    s = system(2500, 12)
    br, lam = 100, 1e-4
    v32 = s["val"].astype(np.float32)
    s32 = dict(s, val=v32.astype(np.float64))
    b = O.residual(s32, np.zeros(s["m"]), -s["xstar"])     # b = A32 x*
    iters = 30
    ref = O.solve(s32, br, lam, b, seed=6, max_iters=iters)
    sol = solver(s, br, lam, values=dev(v32, torch.float32))
    sol.set_replay(ref["tau"], ref["I"], iters)
    x, _ = sol.solve(dev(b, torch.float32), seed=0, tol=0.0, max_iters=iters, replay=True)
    e = rel(host(x), ref["x"])
    print(f"csr fp32 replay rel err {e:.2e}", flush=True)
    assert x.dtype == torch.float32 and e < 1e-4


def test_csr_refine_fp64_inner_is_restart_equivalent():
    """REFINE on FP64 values (inner passes in FP64) reproduces the plain
    solve up to rounding: each outer step restarts ROR-BK on (A, r, 0) with the
    sampler counter continuing."""
    s = system(1800, 12)
    br, lam = 60, 1e-4
    sol = solver(s, br, lam)
    sol.set_refine(7, 0.0)
    b = dev(s["b"])
    x1, _ = sol.solve(b, seed=8, tol=0.0, max_iters=40)
    x2, _ = sol.solve(b, seed=8, tol=0.0, max_iters=40, refine=True)
    e = rel(host(x2), host(x1))
    print(f"csr refine restart equivalence {e:.2e}", flush=True)
    assert e < 1e-9


def test_csr_refine_fp32():
    s = system(2000, 12, scale_lo=0.0)
    br, lam = 50, 1e-4
    v = dev(s["val"])
    sol = solver(s, br, lam, values=v.float(), A64=v)
    b = dev(s["b"])
    x, info = sol.solve(b, seed=2, tol=1e-3, max_iters=300, refine=True)
    r = O.residual(s, s["b"], host(x))
    rrn = np.linalg.norm(r) / np.linalg.norm(s["b"])
    print(f"csr refine fp32: iters {info['iters']} reported rrn {info['rrn']:.2e} FP64 rrn of x "
          f"{rrn:.2e} converged {info['converged']}", flush=True)
    assert x.dtype == torch.float64 and rrn < 1.0
    if info["converged"]:
        assert rrn < 1e-3 * (1 + 1e-6)


def test_csr_backward_matches_oracle():
    s = system(1200, 12)
    br, lam = 40, 1e-3
    iters = 15
    rng = np.random.default_rng(2)
    x0 = rng.standard_normal(s["n"])
    xt = rng.standard_normal(s["n"])
    sol = solver(s, br, lam)
    x, _ = sol.solve(dev(s["b"]), dev(x0), seed=9, tol=0.0, max_iters=iters, record=True)
    rec = sol.record()
    g = 2 * (host(x) - xt)
    gb, gx0 = sol.backward(dev(g))
    rb, rx0 = O.backward(s, br, lam, rec["tau"], rec["I"], iters, False, g)
    eb, ex = rel(host(gb), rb), rel(host(gx0), rx0)
    print(f"csr adjoint: dL/db {eb:.2e}, dL/dx0 {ex:.2e}", flush=True)
    assert eb < 1e-10 and ex < 1e-10


def test_csr_invalid_input_rejected():
    s = system(500, 5)
    colidx = s["colidx"].copy()
    colidx[[3, 4]] = colidx[[4, 3]]          # row 0 no longer ascending
    with pytest.raises(P.RorBkError) as ei:
        P.Solver(None, 25, 1e-3, rowptr=dev(s["rowptr"], torch.int64),
                 colidx=dev(colidx, torch.int32), values=dev(s["val"]),
                 shape=(s["m"], s["n"]))
    assert ei.value.code == P.RORBK_ERR_INVALID_ARG
    rowptr = s["rowptr"].copy()
    rowptr[-1] -= 1                            # rowptr[m] != nnz
    with pytest.raises(P.RorBkError):
        P.Solver(None, 25, 1e-3, rowptr=dev(rowptr, torch.int64),
                 colidx=dev(s["colidx"], torch.int32), values=dev(s["val"]),
                 shape=(s["m"], s["n"]))


@pytest.mark.timeout(600)
def test_csr_full_size():
    """The full sparse workload (200000^2, 2.6M entries, blocks of 128): the
    setup's S for every block, sampled block inverses, and three free-running
    iterations against the oracle."""
    w = make("csr_200000")
    br, lam, seed = w["block_rows"], w["lam"], w["seed"]
    print("csr full size: setup", flush=True)
    sol = solver(w, br, lam)
    got = sol.setup_arrays()
    S = O.cosine_rowsums(w, br)
    np.testing.assert_allclose(got["S"], S, rtol=1e-12)
    off = got["offsets"]
    for t in (0, 777, sol.k - 1):
        rows = np.arange(off[t], off[t + 1])
        L = O.block_factor(w, rows, lam)
        Hinv = np.linalg.inv(L @ L.T)
        assert rel(sol.block_inverse(t), Hinv) < 50 * np.linalg.cond(L @ L.T) * np.finfo(float).eps
    iters = 3
    ref = O.solve(w, br, lam, w["b"], seed=seed, max_iters=iters)
    x, _ = sol.solve(dev(w["b"]), seed=seed, tol=0.0, max_iters=iters, record=True)
    rec = sol.record()
    np.testing.assert_array_equal(rec["tau"], ref["tau"])
    np.testing.assert_array_equal(rec["I"], ref["I"])
    e = rel(host(x), ref["x"])
    print(f"csr full size: {iters} iterations rel err {e:.2e}", flush=True)
    assert e < 1e-10
