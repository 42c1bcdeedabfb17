"""GPU parity of the dense FP64 path against the FP64 oracle.

Bars: integer results (partition, sampled blocks given the same W, top-K given
the same residual, recorded greedy sets) bit-exact; FP64 vectors within the
relative tolerances stated per test (derived from the condition of the block
solves: a few hundred ulps after hundreds of iterations).
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

SHAPES = [
    # m, n, block_rows, lam, cond   (ragged partitions / column tails)
    (1000, 300, 20, 1e-3, 1e4),
    (1037, 257, 16, 1e-4, 1e6),
    (300, 5000, 10, 1e-4, 1e3),
    (2000, 200, 20, 1e-3, 1e6),
    (640, 2100, 64, 1e-4, 1e2),
    (700, 90, 129, 1e-2, 1e3),
]


def make(m, n, cond, cfg=11):
    return dense_svd_system(m, n, cond, cfg=cfg + m + n)


@pytest.mark.parametrize("m,n,br,lam,cond", SHAPES)
def test_setup_matches_oracle(m, n, br, lam, cond):
    s = make(m, n, cond)
    print(f"setup m={m} n={n} br={br}", flush=True)
    A = dev(s["A"])
    sol = P.Solver(A, br, lam)
    got = sol.setup_arrays()
    off = O.partition(m, br)
    np.testing.assert_array_equal(got["offsets"], off)          # bit-exact
    S = O.cosine_rowsums(s["A"], br)
    pbar, W = O.proposal(S, n)
    np.testing.assert_allclose(got["S"], S, rtol=1e-12)
    np.testing.assert_allclose(got["pbar"], pbar, rtol=1e-12)
    np.testing.assert_allclose(got["W"], W, rtol=1e-12)
    # stored inverse of a few blocks vs the oracle's factor
    for t in sorted({0, len(off) // 2, len(off) - 2}):
        rows = np.arange(off[t], off[t + 1])
        L = O.block_factor(s["A"], rows, lam)
        Hinv = np.linalg.inv(L @ L.T)
        Hg = sol.block_inverse(t)
        cond_g = np.linalg.cond(L @ L.T)
        assert rel(Hg, Hinv) < 50 * cond_g * np.finfo(float).eps


@pytest.mark.parametrize("k", [1, 2, 7, 100, 1562, 5000])
def test_sampler_bit_exact(k):
    """Given the same W, the device sampler draws exactly the oracle's blocks."""
    rng = np.random.default_rng(k)
    pbar = rng.uniform(0.0, 1.0, k)
    pbar[rng.integers(0, k, size=max(1, k // 10))] = 0.0
    pbar[0] += 1e-3
    W = np.cumsum(pbar)
    A = rng.standard_normal((2 * k, 16))
    sol = P.Solver(dev(A), 2, 1e-3)
    assert sol.k == k
    sol.set_proposal(W)
    for seed, j0, cnt in [(0, 0, 50), (12345678901234567, 1000, 333), ((1 << 64) - 1, 7, 10)]:
        got = sol.sample(seed, j0, cnt)
        ref = O.sample_many(seed, j0, cnt, W)
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("m,br,dt", [(1000, 20, torch.float64), (5000, 64, torch.float64),
                                     (100000, 64, torch.float64), (3000, 128, torch.float32),
                                     (4099, 129, torch.float64), (200000, 128, torch.float32)])
def test_topk_bit_exact(m, br, dt):
    """Given the same residual, the greedy set equals the oracle's (ties to the
    lower index), for chunked and multi-level selections."""
    rng = np.random.default_rng(m + br)
    A = rng.standard_normal((m, 4))
    sol = P.Solver(dev(A, dt), br, 1e-3)
    K = sol.K
    for trial in range(3):
        r = rng.standard_normal(m) * 10.0 ** rng.uniform(-8, 0, m)
        if trial == 1:   # heavy ties: few distinct magnitudes, both signs
            r = rng.choice([-3.0, -1.0, 0.0, 1.0, 2.0, 3.0], size=m)
        if trial == 2:
            r = np.zeros(m)
        if dt == torch.float32:
            r = r.astype(np.float32).astype(np.float64)
        idx = host(sol.topk(dev(r, dt)))
        np.testing.assert_array_equal(idx, O.topk(r, K))


@pytest.mark.parametrize("m,n,br,lam,cond", SHAPES)
def test_residual_and_block_norms(m, n, br, lam, cond):
    s = make(m, n, cond)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(n)
    sol = P.Solver(dev(s["A"]), br, lam)
    r, bn, rrn = sol.residual(dev(s["b"]), dev(x))
    rr = O.residual(s["A"], s["b"], x)
    scale = np.abs(s["A"]) @ np.abs(x) + np.abs(s["b"])
    assert np.all(np.abs(host(r) - rr) <= 1e-13 * scale + 1e-300)
    off = O.partition(m, br)
    bref = np.array([np.sum(rr[off[t]:off[t + 1]] ** 2) for t in range(len(off) - 1)])
    np.testing.assert_allclose(host(bn), bref, rtol=1e-11)
    assert rrn == pytest.approx(np.linalg.norm(rr) / np.linalg.norm(s["b"]), rel=1e-12)


@pytest.mark.parametrize("m,n,br,lam,cond", SHAPES)
def test_replay_trajectory_fp64(m, n, br, lam, cond):
    """Replay the oracle's tau and greedy sets: x within 1e-10 relative."""
    s = make(m, n, cond)
    iters = 60
    ref = O.solve(s["A"], br, lam, s["b"], seed=5, max_iters=iters)
    sol = P.Solver(dev(s["A"]), br, lam)
    sol.set_replay(ref["tau"], ref["I"], iters)
    b = dev(s["b"])
    x, info = sol.solve(b, seed=0, tol=0.0, max_iters=iters, replay=True, record=True)
    assert info["iters"] == iters and not info["converged"]
    e = rel(host(x), ref["x"])
    print(f"replay m={m} n={n} br={br}: rel err {e:.3e}", flush=True)
    assert e < 1e-10
    rec = sol.record()
    np.testing.assert_array_equal(rec["tau"], ref["tau"])
    np.testing.assert_array_equal(rec["I"], ref["I"])
    np.testing.assert_allclose(rec["rrn"], ref["rrn_hist"], rtol=1e-9)


# Greedy sets at the edges of the panel solve's padded sizes (16, 32 and 64
# rows: sets of 17, 32, 33, 48 and 63 rows) through the chain form's greedy
# solve, replayed against the oracle.
@pytest.mark.parametrize("m,n,br", [(17 * 40, 300, 17), (32 * 40, 300, 32), (33 * 40, 257, 33),
                                    (48 * 30, 400, 48), (63 * 30, 500, 63)])
def test_replay_greedy_set_sizes(m, n, br):
    s = make(m, n, 1e3)
    iters = 40
    ref = O.solve(s["A"], br, 1e-3, s["b"], seed=6, max_iters=iters)
    sol = P.Solver(dev(s["A"]), br, 1e-3)
    assert sol.K == br
    sol.set_replay(ref["tau"], ref["I"], iters)
    x, info = sol.solve(dev(s["b"]), seed=0, tol=0.0, max_iters=iters, replay=True)
    e = rel(host(x), ref["x"])
    print(f"replay K={br}: rel err {e:.3e}", flush=True)
    assert e < 1e-10


@pytest.mark.parametrize("m,n,br,lam,cond", SHAPES[:4])
def test_free_running_matches_oracle(m, n, br, lam, cond):
    """Free running with the oracle's W: identical draws and greedy sets."""
    s = make(m, n, cond)
    iters = 40
    ref = O.solve(s["A"], br, lam, s["b"], seed=77, max_iters=iters)
    sol = P.Solver(dev(s["A"]), br, lam)
    _, Wref = O.proposal(O.cosine_rowsums(s["A"], br), n)
    sol.set_proposal(Wref)
    x, info = sol.solve(dev(s["b"]), seed=77, tol=0.0, max_iters=iters, record=True)
    rec = sol.record()
    np.testing.assert_array_equal(rec["tau"], ref["tau"])
    np.testing.assert_array_equal(rec["I"], ref["I"])
    assert rel(host(x), ref["x"]) < 1e-10


MULTI_SLAB = [
    (400, 9001, 16),    # FP64 3 rows per thread (prefetch), odd n misaligns FP64 rows
    (420, 8960, 20),
    (1000, 8704, 50),   # FP64 9 rows per thread with the prefetch
    (1100, 8400, 100),  # FP64 21 rows per thread, no prefetch; greedy set of 100 rows
]


@pytest.mark.parametrize("m,n,br", MULTI_SLAB)
@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_multi_slab_update_workgroups(m, n, br, storage):
    """More than 64 slabs of 128 columns: each update workgroup takes two and
    loads the second while the first is reduced (ragged last slab; odd n also
    misaligns the FP64 rows).  The block sizes cover each rows-per-thread
    instantiation of the step kernel.  FP64 storage against the oracle;
    FP32 and BF16 storage replayed on the oracle's draws and greedy sets
    against the oracle run on the rounded matrix."""
    s = make(m, n, 1e3)
    lam = 1e-4
    iters = 20
    if storage == "f64":
        A = s["A"]
        ref = O.solve(A, br, lam, s["b"], seed=31, max_iters=iters)
        sol = P.Solver(dev(A), br, lam)
        _, Wref = O.proposal(O.cosine_rowsums(A, br), n)
        sol.set_proposal(Wref)
        x, _ = sol.solve(dev(s["b"]), seed=31, tol=0.0, max_iters=iters, record=True)
        rec = sol.record()
        np.testing.assert_array_equal(rec["tau"], ref["tau"])
        np.testing.assert_array_equal(rec["I"], ref["I"])
        e = rel(host(x), ref["x"])
        print(f"multi-slab f64 m={m} n={n}: rel err {e:.2e}", flush=True)
        assert e < 1e-10
    else:
        if storage == "f32":
            Av = s["A"].astype(np.float32).astype(np.float64)
            At = dev(s["A"], torch.float32)
        else:
            Av = bf16_values(s["A"])
            At = bf16_tensor(s["A"])
        b = Av @ s["xstar"]
        ref = O.solve(Av, br, lam, b, seed=31, max_iters=iters)
        sol = P.Solver(At, br, lam)
        sol.set_replay(ref["tau"], ref["I"], iters)
        x, _ = sol.solve(dev(b, torch.float32), seed=0, tol=0.0, max_iters=iters, replay=True)
        assert x.dtype == torch.float32
        e = rel(host(x), ref["x"])
        print(f"multi-slab {storage} m={m} n={n} br={br}: rel err vs FP64 oracle {e:.2e}",
              flush=True)
        assert e < 1e-4


def test_selection_chunks_of_many_segments():
    """n = 16385 columns (9 column segments of the residual pass): the
    selection splits the 1200 rows into chunks of at most 8192 partial
    products (906 and 294 rows, both shorter than a full set of rounds),
    sums the 9 segments in groups of four loads and merges the two candidate
    lists.  FP64 trajectory against the oracle (draws and greedy sets
    bit-exact) and the top-K of given residuals bit-exact."""
    rng = np.random.default_rng(7)
    m, n, br, lam, iters = 1200, 16385, 6, 1e-3, 15
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    b = A @ rng.standard_normal(n)
    ref = O.solve(A, br, lam, b, seed=5, max_iters=iters)
    sol = P.Solver(dev(A), br, lam)
    _, Wref = O.proposal(O.cosine_rowsums(A, br), n)
    sol.set_proposal(Wref)
    x, _ = sol.solve(dev(b), seed=5, tol=0.0, max_iters=iters, record=True)
    rec = sol.record()
    np.testing.assert_array_equal(rec["tau"], ref["tau"])
    np.testing.assert_array_equal(rec["I"], ref["I"])
    e = rel(host(x), ref["x"])
    print(f"many-segment selection: rel err {e:.2e}", flush=True)
    assert e < 1e-10
    for trial in range(2):
        r = rng.standard_normal(m) * 10.0 ** rng.uniform(-8, 0, m)
        if trial == 1:   # ties
            r = rng.choice([-2.0, 0.0, 1.0, 2.0], size=m)
        np.testing.assert_array_equal(host(sol.topk(dev(r))), O.topk(r, sol.K))


def test_stop_test_and_iteration_count():
    s = make(1000, 300, 1e4)
    ref = O.solve(s["A"], 20, 1e-3, s["b"], seed=9, tol=0.05, max_iters=500)
    assert ref["converged"]
    sol = P.Solver(dev(s["A"]), 20, 1e-3)
    _, Wref = O.proposal(O.cosine_rowsums(s["A"], 20), 300)
    sol.set_proposal(Wref)
    x, info = sol.solve(dev(s["b"]), seed=9, tol=0.05, max_iters=500)
    assert info["converged"] and info["iters"] == ref["iters"]
    assert info["rrn"] == pytest.approx(ref["rrn"], rel=1e-9)
    assert rel(host(x), ref["x"]) < 1e-10


def test_resume_matches_full_run():
    """A solve resumed at iteration 20 from the iterate a 20-iteration solve
    returned follows the same selections as one 50-iteration solve.  Within a
    solve the fused step of iteration it also takes the sampled steps of
    it + 1 (their z from the residual and A_{S'} A_I^T); a resumed solve starts
    those from x, so the two iterates agree to rounding, not bit for bit.
    Repeated solves are bit-identical."""
    s = make(1000, 300, 1e4)
    sol = P.Solver(dev(s["A"]), 20, 1e-3)
    b = dev(s["b"])
    x_full, _ = sol.solve(b, seed=3, tol=0.0, max_iters=50, record=True)
    I_full = sol.record()["I"]
    x_half, _ = sol.solve(b, seed=3, tol=0.0, max_iters=20, record=True)
    I_half = sol.record()["I"]
    x_rest, _ = sol.solve(b, x_half, seed=3, tol=0.0, max_iters=30, start_iter=20, record=True)
    I_rest = sol.record()["I"]
    assert np.array_equal(np.concatenate([I_half, I_rest]), I_full)
    assert (torch.linalg.norm(x_rest - x_full) / torch.linalg.norm(x_full)).item() < 1e-12
    x_again, _ = sol.solve(b, seed=3, tol=0.0, max_iters=50)
    assert torch.equal(x_full, x_again)          # deterministic


def test_errors():
    s = make(200, 30, 1e2)
    b = s["b"].copy()
    b[7] = np.nan
    sol = P.Solver(dev(s["A"]), 10, 1e-3)
    with pytest.raises(P.RorBkError) as e:
        sol.solve(dev(b), seed=1, tol=0.0, max_iters=5)
    assert e.value.code == P.RORBK_ERR_NONFINITE
    A0 = s["A"].copy()
    A0[13] = 0.0
    with pytest.raises(P.RorBkError) as e:
        P.Solver(dev(A0), 10, 0.0)
    assert e.value.code == P.RORBK_ERR_NOT_SPD
    with pytest.raises(P.RorBkError) as e:
        P.Solver(dev(s["A"]), 500, 1e-3)
    assert e.value.code == P.RORBK_ERR_INVALID_ARG
    with pytest.raises(P.RorBkError) as e:
        P.Solver(dev(s["A"]), 10, -1.0)
    assert e.value.code == P.RORBK_ERR_INVALID_ARG
    with pytest.raises(P.RorBkError) as e:
        sol.backward(dev(np.zeros(30)))
    assert e.value.code == P.RORBK_ERR_NOT_RECORDED


def test_info_rrn_is_that_of_the_returned_iterate():
    """rorbk_info.rrn is ||b - A x|| / ||b|| of the x returned: after a solve
    that ends at its cap (one greedy update after the last stop test) it is
    measured again; rrn_test keeps the last stop test, which the RRN history
    ends with; t_setup_s reports the setup's wall time."""
    s = make(1000, 300, 1e4)
    sol = P.Solver(dev(s["A"]), 20, 1e-3)
    b = dev(s["b"])
    x, info = sol.solve(b, seed=9, tol=0.0, max_iters=25, record=True)
    rr = np.linalg.norm(s["b"] - s["A"] @ host(x)) / np.linalg.norm(s["b"])
    assert not info["converged"]
    assert info["rrn"] == pytest.approx(rr, rel=1e-10)
    hist = sol.record()["rrn"]
    assert info["rrn_test"] == pytest.approx(hist[-1], rel=1e-14)
    assert 0.0 < info["t_setup_s"] < 60.0
    # a converged solve returns the tested iterate: both fields agree
    x2, i2 = sol.solve(b, seed=9, tol=0.2, max_iters=500)
    assert i2["converged"] and i2["rrn"] == i2["rrn_test"] < 0.2
    rr2 = np.linalg.norm(s["b"] - s["A"] @ host(x2)) / np.linalg.norm(s["b"])
    assert i2["rrn"] == pytest.approx(rr2, rel=1e-10)


def test_record_of_a_later_solve_without_greedy_sets_is_refused():
    """A solve that does not record its greedy sets replaces the record: the
    sets of an older recorded solve are not returned any more."""
    s = make(600, 120, 1e3)
    sol = P.Solver(dev(s["A"]), 20, 1e-3)
    b = dev(s["b"])
    sol.solve(b, seed=3, tol=0.0, max_iters=30, record=True)
    rec = sol.record()
    assert rec["iters"] == 30 and rec["I"] is not None
    sol.solve(b, seed=4, tol=0.0, max_iters=20)          # not recorded
    rec2 = sol.record()
    assert rec2["iters"] == 20 and rec2["I"] is None
    with pytest.raises(P.RorBkError) as e:
        sol.backward(torch.ones(120, dtype=torch.float64, device="cuda:0"))
    assert e.value.code == P.RORBK_ERR_NOT_RECORDED
