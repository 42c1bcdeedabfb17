"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them retypes the oracle's own
formula: they use closed forms, textbook special cases, identities proved in
the paper, invariants, brute force with different primitives (numpy solves,
sorts) and published test vectors.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
from tests.conftest import read_golden
from workloads import dense_svd_system, csr_system, WORKLOADS


def rand_dense(rng, m, n):
    return rng.standard_normal((m, n))


# --------------------------------------------------------------- partition --

@pytest.mark.parametrize("m", [1, 2, 7, 10, 37, 100, 257])
def test_partition_structure(m):
    """Algorithm 1, first step: k contiguous blocks, each >= floor(m/k) rows."""
    for b in range(1, m + 1):
        off = O.partition(m, b)
        k = len(off) - 1
        assert k == m // b
        sizes = np.diff(off)
        q = m // k
        assert off[0] == 0 and off[-1] == m           # covers all rows, contiguous
        assert np.all(sizes >= q) and np.all(sizes <= q + 1)
        # the extra rows go to the first blocks (array_split reading)
        ref = [len(s) for s in np.array_split(np.arange(m), k)]
        assert sizes.tolist() == ref


def test_partition_workloads():
    """Block counts and remainders of the five workloads."""
    expect = {"dense_2000x200": (100, 0), "tall_100000x2000": (1562, 32),
              "csr_200000": (1562, 64), "wide_2000x50000": (62, 16),
              "diff_20000x1000": (400, 0)}
    for name, (k, rem) in expect.items():
        w = WORKLOADS[name]
        off = O.partition(w["m"], w["block_rows"])
        sizes = np.diff(off)
        assert len(sizes) == k
        assert int(np.sum(sizes == sizes.min() + 1)) == rem


def test_partition_rejects_bad_sizes():
    assert O.num_blocks(10, 0) == 0
    assert O.num_blocks(10, 11) == 0
    with pytest.raises(O.OracleError):
        O.partition(10, 11)


# ---------------------------------------------------------------- proposal --

def test_proposal_three_block_hand_example(golden_dir):
    """Section 2 proposal equation on a hand-worked 3-block example."""
    g = read_golden(os.path.join(golden_dir, "proposal_three_blocks.txt"))
    r3 = math.sqrt(3.0)
    A = np.array([[1, 0], [0.5, 0],
                  [0.25, r3 / 4], [0.25, r3 / 4],
                  [0, 2], [0, 1]], dtype=np.float64)
    S = O.cosine_rowsums(A, 2)
    np.testing.assert_allclose(S, [float(v) for v in g["S"]], rtol=2e-15)
    pbar, W = O.proposal(S, 2)
    np.testing.assert_allclose(pbar, [float(v) for v in g["Pbar"]], rtol=2e-15)
    np.testing.assert_allclose(np.diff(np.concatenate([[0], W])) / W[-1],
                               [float(v) for v in g["P"]], rtol=2e-15)


def test_proposal_block_orthogonal_is_uniform(rng):
    """Disjoint column supports -> C = I -> S_t = 1 -> P uniform."""
    k, rows, w = 6, 3, 4
    A = np.zeros((k * rows, k * w))
    for t in range(k):
        A[t * rows:(t + 1) * rows, t * w:(t + 1) * w] = rng.standard_normal((rows, w))
    S = O.cosine_rowsums(A, rows)
    np.testing.assert_allclose(S, np.ones(k), rtol=0, atol=1e-15)
    pbar, W = O.proposal(S, A.shape[1])
    np.testing.assert_allclose(pbar, math.exp(-2.0 / A.shape[1]), rtol=1e-15)
    np.testing.assert_allclose(W, np.arange(1, k + 1) * pbar[0], rtol=1e-14)


def test_proposal_parallel_blocks_is_uniform(rng):
    """All rows equal -> every centroid parallel -> C = ones -> S_t = k."""
    row = rng.standard_normal(5)
    A = np.tile(row, (12, 1))
    S = O.cosine_rowsums(A, 3)
    np.testing.assert_allclose(S, np.full(4, 4.0), rtol=1e-15)


def test_proposal_zero_centroid():
    """A block whose rows cancel has a zero centroid: C(t,t)=1, C(t,j)=0."""
    A = np.array([[1.0, 2.0], [-1.0, -2.0], [1.0, 0.0], [0.0, 1.0]])
    S = O.cosine_rowsums(A, 2)
    c = 1.0 / math.sqrt(2.0)       # centroid of block 1 is (1,1); block 0 is zero
    np.testing.assert_allclose(S, [1.0, 1.0], atol=1e-15)
    A2 = np.array([[1.0, 0.0], [0.0, 1.0], [2.0, 0.0], [0.0, 0.0]])
    S2 = O.cosine_rowsums(A2, 2)  # centroids (1,1) and (2,0): cos = 1/sqrt2
    np.testing.assert_allclose(S2, [1 + c, 1 + c], rtol=1e-15)


@pytest.mark.parametrize("m,n,b", [(12, 5, 3), (30, 8, 4), (9, 20, 2), (40, 3, 7)])
def test_proposal_brute_force(rng, m, n, b):
    """Centroid cosines by numpy (reduceat sums, normalised Gram)."""
    A = rand_dense(rng, m, n)
    off = np.array([len(s) for s in np.array_split(np.arange(m), m // b)]).cumsum()
    starts = np.concatenate([[0], off[:-1]])
    cen = np.add.reduceat(A, starts, axis=0)
    un = cen / np.linalg.norm(cen, axis=1, keepdims=True)
    C = np.abs(un @ un.T)
    S = O.cosine_rowsums(A, b)
    np.testing.assert_allclose(S, C.sum(axis=1), rtol=1e-13)
    pbar, W = O.proposal(S, n)
    np.testing.assert_allclose(pbar, np.exp(-2 * C.sum(axis=1) / n), rtol=1e-13)
    np.testing.assert_allclose(W, np.cumsum(pbar), rtol=1e-14)


def test_proposal_csr_matches_dense(rng):
    """The sparse centroid path agrees with the dense one on the same matrix."""
    sysd = csr_system(300, 5, cfg=77)
    M = O.Matrix(sysd)
    S_csr = O.cosine_rowsums(sysd, 16)
    S_dense = O.cosine_rowsums(M.dense(), 16)
    np.testing.assert_allclose(S_csr, S_dense, rtol=1e-13)
    part = O.cosine_rowsums(sysd, 16, 3, 9)
    np.testing.assert_array_equal(part, S_csr[3:9])


# ----------------------------------------------------------------- sampler --

def test_splitmix64_published_vector(golden_dir):
    g = read_golden(os.path.join(golden_dir, "splitmix64_seed0.txt"))
    for c in range(4):
        assert O.splitmix64_word(0, c) == int(g[f"word{c}"][0], 16)


def test_sampler_distribution_chi2():
    """Draws follow P = Pbar / sum(Pbar): chi-square goodness of fit."""
    from scipy.stats import chisquare
    pbar = np.array([0.5, 0.1, 0.0, 0.25, 0.9, 0.05, 0.3])
    W = np.cumsum(pbar)
    draws = O.sample_many(2024, 0, 40000, W)          # 120000 draws
    counts = np.bincount(draws, minlength=len(pbar))
    assert counts[2] == 0                              # zero-probability block
    keep = pbar > 0
    exp = pbar[keep] / pbar.sum() * draws.size
    assert chisquare(counts[keep], exp).pvalue > 1e-4


def test_sampler_single_block_and_determinism():
    assert all(O.sample(s, j, l, np.array([0.3])) == 0
               for s in (0, 1, 99) for j in range(5) for l in (1, 2, 3))
    W = np.cumsum(np.linspace(0.1, 1.0, 50))
    a = O.sample_many(7, 100, 50, W)
    b = O.sample_many(7, 100, 50, W)
    np.testing.assert_array_equal(a, b)
    # draw l of iteration j is stream word 3j + l - 1: iteration 101 of a run
    # started at 100 equals iteration 1 of a run started at 100 - 100 + 101
    c = O.sample_many(7, 101, 49, W)
    np.testing.assert_array_equal(a[3:], c)


# -------------------------------------------------------------- small solve --

@pytest.mark.parametrize("K", [1, 2, 5, 17, 64, 129])
def test_cholesky_vs_numpy(rng, K):
    B = rng.standard_normal((K, K + 3))
    G = B @ B.T + 1e-3 * np.eye(K)
    L = O.cholesky(G)
    np.testing.assert_allclose(L, np.linalg.cholesky(G), rtol=1e-10, atol=1e-12)
    r = rng.standard_normal(K)
    np.testing.assert_allclose(O.chol_solve(L, r), np.linalg.solve(G, r), rtol=1e-8)


def test_cholesky_detects_non_spd():
    with pytest.raises(O.OracleError) as e:
        O.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert e.value.code == O.ORC_ERR_NOT_SPD
    # a zero row with mu = 0 makes the block Gram singular
    A = np.array([[1.0, 0.0], [0.0, 0.0]])
    with pytest.raises(O.OracleError):
        O.block_factor(A, [0, 1], 0.0)


# -------------------------------------------------------------- block update --

def test_kaczmarz_special_case(rng):
    """One row, mu = 0 reduces to the classical Kaczmarz projection
    (Section 2, the single-row update) and zeroes that row's residual."""
    A = rand_dense(rng, 9, 6)
    b = rng.standard_normal(9)
    x = rng.standard_normal(6)
    for i in range(9):
        xn = O.apply_block(A, [i], 0.0, b, x)
        kac = x + (b[i] - A[i] @ x) / (A[i] @ A[i]) * A[i]
        np.testing.assert_allclose(xn, kac, rtol=1e-13, atol=1e-14)
        assert abs(b[i] - A[i] @ xn) <= 16 * np.finfo(float).eps * (
            np.linalg.norm(A[i]) * np.linalg.norm(xn) + abs(b[i]))


def test_motzkin_special_case(rng):
    """Block size 1: the greedy row is the one of largest |r_i| (Motzkin)."""
    A = rand_dense(rng, 15, 4)
    b = rng.standard_normal(15)
    out = O.solve(A, 1, 1e-12, b, seed=3, max_iters=4)
    x = np.zeros(4)
    for it in range(4):
        for l in range(3):
            x = O.apply_block(A, [out["tau"][3 * it + l]], 1e-12, b, x)
        r = b - A @ x
        assert out["I"][it][0] == int(np.argmax(np.abs(r)))
        x = O.apply_block(A, out["I"][it], 1e-12, b, x)
    np.testing.assert_allclose(out["x"], x, rtol=1e-10)


def test_one_block_is_regularized_least_squares(rng):
    """k = 1: each update is the closed-form regularised LS step
    x+ = (A^T A + mu I)^{-1}(A^T b + mu x)  (Lemma 1), checked with lstsq on
    the stacked system [A; sqrt(mu) I] x = [b; sqrt(mu) x]."""
    m, n, mu = 8, 12, 0.3
    A = rand_dense(rng, m, n)
    b = rng.standard_normal(m)
    x0 = rng.standard_normal(n)
    out = O.solve(A, m, mu, b, x0=x0, seed=1, max_iters=2)
    x = x0.copy()
    for _ in range(8):             # 2 iterations x (3 sampled + 1 greedy) steps
        M = np.vstack([A, math.sqrt(mu) * np.eye(n)])
        rhs = np.concatenate([b, math.sqrt(mu) * x])
        x = np.linalg.lstsq(M, rhs, rcond=None)[0]
    np.testing.assert_allclose(out["x"], x, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("rows,n", [(3, 10), (10, 4), (6, 6)])
def test_update_identities(rng, rows, n):
    """Lemma 1 (row form = column form), the block-residual identity
    b_S - A_S x+ = mu (A_S A_S^T + mu I)^{-1} (b_S - A_S x), and Theorem 1's
    exact error relation e+ = mu (A_S^T A_S + mu I)^{-1} e with
    ||e+|| <= ||e|| on a consistent system."""
    m, mu = 20, 0.05
    A = rand_dense(rng, m, n)
    xs = rng.standard_normal(n)
    b = A @ xs
    x = rng.standard_normal(n)
    S = np.arange(4, 4 + rows)
    xn = O.apply_block(A, S, mu, b, x)
    AS = A[S]
    col = x + np.linalg.solve(AS.T @ AS + mu * np.eye(n), AS.T @ (b[S] - AS @ x))
    np.testing.assert_allclose(xn, col, rtol=1e-10, atol=1e-12)
    r_new = b[S] - AS @ xn
    r_old = b[S] - AS @ x
    np.testing.assert_allclose(r_new, mu * np.linalg.solve(AS @ AS.T + mu * np.eye(rows), r_old),
                               rtol=1e-9, atol=1e-12)
    e_new = xn - xs
    np.testing.assert_allclose(e_new, mu * np.linalg.solve(AS.T @ AS + mu * np.eye(n), x - xs),
                               rtol=1e-9, atol=1e-12)
    assert np.linalg.norm(e_new) <= np.linalg.norm(x - xs) * (1 + 1e-14)


def test_csr_update_matches_dense(rng):
    sysd = csr_system(60, 4, cfg=91)
    M = O.Matrix(sysd)
    D = M.dense()
    x = rng.standard_normal(60)
    S = [3, 17, 18, 40, 59]
    np.testing.assert_allclose(O.apply_block(sysd, S, 1e-3, sysd["b"], x),
                               O.apply_block(D, S, 1e-3, sysd["b"], x), rtol=1e-12)
    np.testing.assert_allclose(O.residual(sysd, sysd["b"], x),
                               sysd["b"] - D @ x, rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------------- top-K --

def test_topk_brute_force(rng):
    for m, K in [(1, 1), (10, 3), (100, 20), (1000, 64), (513, 129)]:
        r = rng.standard_normal(m) * 10.0 ** rng.uniform(-6, 0, m)
        idx = O.topk(r, K)
        ref = np.sort(np.lexsort((np.arange(m), -np.abs(r)))[:K])
        np.testing.assert_array_equal(idx, ref)


def test_topk_ties_go_to_lower_index():
    r = np.array([1.0, -3.0, 3.0, 2.0, -3.0, 0.0, 3.0])
    np.testing.assert_array_equal(O.topk(r, 2), [1, 2])
    np.testing.assert_array_equal(O.topk(r, 4), [1, 2, 4, 6])
    np.testing.assert_array_equal(O.topk(np.zeros(5), 2), [0, 1])


def test_topk_nan_is_an_error():
    with pytest.raises(O.OracleError) as e:
        O.topk(np.array([1.0, np.nan, 2.0]), 1)
    assert e.value.code == O.ORC_ERR_NONFINITE


# -------------------------------------------------------------- whole solve --

def brute_force_solve(A, b, block_rows, mu, taus, iters, x0=None):
    """Algorithm 1 with numpy primitives: dense solves and an argsort top-K."""
    m, n = A.shape
    k = m // block_rows
    K = m // k
    bounds = np.concatenate([[0], np.cumsum([len(s) for s in np.array_split(np.arange(m), k)])])
    x = np.zeros(n) if x0 is None else x0.copy()
    Is = []
    for it in range(iters):
        for l in range(3):
            t = taus[3 * it + l]
            rows = np.arange(bounds[t], bounds[t + 1])
            As = A[rows]
            x = x + As.T @ np.linalg.solve(As @ As.T + mu * np.eye(len(rows)), b[rows] - As @ x)
        r = b - A @ x
        order = sorted(range(m), key=lambda i: (-abs(r[i]), i))
        I = np.array(sorted(order[:K]))
        Is.append(I)
        As = A[I]
        x = x + As.T @ np.linalg.solve(As @ As.T + mu * np.eye(K), r[I])
    return x, np.array(Is)


@pytest.mark.parametrize("m,n,br", [(12, 5, 3), (10, 12, 2), (12, 12, 4), (11, 7, 1)])
def test_solve_brute_force_tiny(rng, m, n, br):
    A = rand_dense(rng, m, n)
    b = A @ rng.standard_normal(n)
    mu = 1e-2
    out = O.solve(A, br, mu, b, seed=5, max_iters=6)
    xb, Ib = brute_force_solve(A, b, br, mu, out["tau"], 6)
    np.testing.assert_array_equal(out["I"], Ib)
    np.testing.assert_allclose(out["x"], xb, rtol=1e-9, atol=1e-11)
    # the recorded tau are the sampler's draws
    k = len(O.partition(m, br)) - 1
    S = O.cosine_rowsums(A, br)
    _, W = O.proposal(S, n)
    np.testing.assert_array_equal(out["tau"], O.sample_many(5, 0, 6, W))
    assert k >= 1


def test_solve_replay_reproduces_free_run(rng):
    A = rand_dense(rng, 40, 9)
    b = A @ rng.standard_normal(9)
    a = O.solve(A, 5, 1e-3, b, seed=11, max_iters=20)
    c = O.solve(A, 5, 1e-3, b, seed=999, max_iters=20,
                replay_tau=a["tau"], replay_I=a["I"].reshape(-1))
    np.testing.assert_array_equal(a["x"], c["x"])


def test_resume_is_bit_exact(rng):
    A = rand_dense(rng, 60, 10)
    b = A @ rng.standard_normal(10)
    full = O.solve(A, 6, 1e-3, b, seed=4, max_iters=30)
    first = O.solve(A, 6, 1e-3, b, seed=4, max_iters=12)
    rest = O.solve(A, 6, 1e-3, b, x0=first["x"], seed=4, max_iters=18, start_iter=12)
    np.testing.assert_array_equal(full["x"], rest["x"])
    np.testing.assert_array_equal(full["tau"], np.concatenate([first["tau"], rest["tau"]]))


def test_restart_equivalence(rng):
    """Block Kaczmarz on (A, b - A x0) from 0 equals (A, b) from x0 with the
    same selections (refinement changes only where rounding enters)."""
    A = rand_dense(rng, 50, 8)
    b = A @ rng.standard_normal(8)
    x0 = rng.standard_normal(8)
    a = O.solve(A, 5, 1e-3, b, x0=x0, seed=8, max_iters=15)
    d = O.solve(A, 5, 1e-3, b - A @ x0, seed=8, max_iters=15,
                replay_tau=a["tau"], replay_I=a["I"].reshape(-1))
    np.testing.assert_allclose(x0 + d["x"], a["x"], rtol=1e-11, atol=1e-12)


def test_stop_test_before_greedy(rng):
    A = rand_dense(rng, 30, 5)
    b = A @ rng.standard_normal(5)
    out = O.solve(A, 5, 1e-3, b, seed=2, tol=10.0, max_iters=50)
    assert out["converged"] and out["iters"] == 1
    # the returned x is the one after the three sampled updates only
    x = np.zeros(5)
    off = O.partition(30, 5)
    for t in out["tau"][:3]:
        x = O.apply_block(A, np.arange(off[t], off[t + 1]), 1e-3, b, x)
    np.testing.assert_allclose(out["x"], x, rtol=1e-13)
    assert out["rrn"] == pytest.approx(np.linalg.norm(b - A @ x) / np.linalg.norm(b), rel=1e-12)
    # tol = 0 never stops
    z = O.solve(A, 5, 1e-3, b, seed=2, tol=0.0, max_iters=7)
    assert not z["converged"] and z["iters"] == 7


def test_convergence_planted_solution():
    """Consistent well-conditioned system: the error to x_star decays."""
    sysd = dense_svd_system(400, 30, 10.0, cfg=31)
    out = O.solve(sysd, 10, 1e-5, sysd["b"], seed=1, tol=1e-10, max_iters=400)
    assert out["converged"]
    re = np.linalg.norm(out["x"] - sysd["xstar"]) / np.linalg.norm(sysd["xstar"])
    assert re < 1e-8


def test_range_space_invariant():
    """Lemma 2: from x0 = 0 every iterate stays in R(A^T); on a consistent
    wide system it approaches the minimum-norm solution."""
    sysd = dense_svd_system(40, 200, 10.0, cfg=41, rowspace=True)
    A = sysd["A"]
    Q, _ = np.linalg.qr(A.T)
    for iters in (1, 5, 40):
        out = O.solve(sysd, 4, 1e-6, sysd["b"], seed=3, max_iters=iters)
        x = out["x"]
        null_part = x - Q @ (Q.T @ x)
        assert np.linalg.norm(null_part) <= 1e-12 * np.linalg.norm(x)
    out = O.solve(sysd, 4, 1e-6, sysd["b"], seed=3, tol=1e-12, max_iters=3000)
    re = np.linalg.norm(out["x"] - sysd["xstar"]) / np.linalg.norm(sysd["xstar"])
    assert re < 1e-6


def test_nonfinite_rhs_is_an_error(rng):
    A = rand_dense(rng, 12, 4)
    b = rng.standard_normal(12)
    b[3] = np.nan
    with pytest.raises(O.OracleError) as e:
        O.solve(A, 3, 1e-3, b, seed=1, max_iters=3)
    assert e.value.code == O.ORC_ERR_NONFINITE


def test_csr_solve_matches_dense():
    sysd = csr_system(120, 6, cfg=5)
    D = O.Matrix(sysd).dense()
    a = O.solve(sysd, 8, 1e-5, sysd["b"], seed=9, max_iters=25)
    c = O.solve(D, 8, 1e-5, sysd["b"], seed=9, max_iters=25)
    np.testing.assert_array_equal(a["tau"], c["tau"])
    np.testing.assert_array_equal(a["I"], c["I"])
    np.testing.assert_allclose(a["x"], c["x"], rtol=1e-10, atol=1e-12)


# ----------------------------------------------------------------- adjoint --

def jacobian_by_replay(A, br, mu, out, x0_dim):
    """Columns of the linear map (x0, b) -> x_K with the selections fixed."""
    m, n = A.shape
    tau, I = out["tau"], out["I"].reshape(-1)
    its = out["iters"]
    full = its - 1 if out["converged"] else its
    off = O.partition(m, br)
    cols = []
    for e in np.eye(n + m):
        x = e[:n]
        if full > 0:
            x = O.solve(A, br, mu, e[n:], x0=x, seed=0, max_iters=full,
                        replay_tau=tau, replay_I=I, record=False)["x"]
        if out["converged"]:       # the stopping iteration has no greedy step
            for t in tau[3 * full:3 * full + 3]:
                x = O.apply_block(A, np.arange(off[t], off[t + 1]), mu, e[n:], x)
        cols.append(x)
    J = np.array(cols).T
    return J[:, :n], J[:, n:]


def test_adjoint_matches_brute_force_jacobian(rng):
    m, n, br, mu = 12, 6, 3, 1e-2
    A = rand_dense(rng, m, n)
    b = rng.standard_normal(m)
    x0 = rng.standard_normal(n)
    out = O.solve(A, br, mu, b, x0=x0, seed=13, max_iters=5)
    Jx, Jb = jacobian_by_replay(A, br, mu, out, n)
    np.testing.assert_allclose(Jx @ x0 + Jb @ b, out["x"], rtol=1e-10, atol=1e-12)
    w = rng.standard_normal(n)
    gb, gx0 = O.backward(A, br, mu, out["tau"], out["I"], out["iters"], out["converged"], w)
    np.testing.assert_allclose(gb, Jb.T @ w, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gx0, Jx.T @ w, rtol=1e-9, atol=1e-12)


def test_adjoint_converged_run_skips_last_greedy(rng):
    m, n, br, mu = 12, 6, 3, 1e-2
    A = rand_dense(rng, m, n)
    b = A @ rng.standard_normal(n)
    out = O.solve(A, br, mu, b, seed=13, tol=0.9, max_iters=50)
    assert out["converged"]
    Jx, Jb = jacobian_by_replay(A, br, mu, out, n)
    # replaying a converged run stops at the same point (same residual test)
    w = rng.standard_normal(n)
    gb, gx0 = O.backward(A, br, mu, out["tau"], out["I"], out["iters"], True, w)
    np.testing.assert_allclose(gb, Jb.T @ w, rtol=1e-9, atol=1e-12)


def test_adjoint_finite_differences(rng):
    """L = ||x_K - x_t||^2 is quadratic in (b, x0) once selections are fixed,
    so central differences are exact up to rounding."""
    m, n, br, mu = 40, 10, 5, 1e-3
    A = rand_dense(rng, m, n)
    b = rng.standard_normal(m)
    x0 = rng.standard_normal(n)
    xt = rng.standard_normal(n)
    out = O.solve(A, br, mu, b, x0=x0, seed=21, max_iters=8)
    tau, I = out["tau"], out["I"].reshape(-1)

    def loss(bb, xx):
        r = O.solve(A, br, mu, bb, x0=xx, seed=0, max_iters=8, replay_tau=tau,
                    replay_I=I, record=False)
        return float(np.sum((r["x"] - xt) ** 2))

    gb, gx0 = O.backward(A, br, mu, tau, out["I"], 8, False, 2 * (out["x"] - xt))
    h = 1e-3
    for i in [0, 7, 19, 39]:
        e = np.zeros(m); e[i] = h
        fd = (loss(b + e, x0) - loss(b - e, x0)) / (2 * h)
        assert fd == pytest.approx(gb[i], rel=1e-7, abs=1e-9)
    for i in [0, 4, 9]:
        e = np.zeros(n); e[i] = h
        fd = (loss(b, x0 + e) - loss(b, x0 - e)) / (2 * h)
        assert fd == pytest.approx(gx0[i], rel=1e-7, abs=1e-9)


# ------------------------------------------------ Algorithm 2 (initial solution)

def test_initial_solution_identity_closed_form():
    """A = I: the row sum is the all-ones vector, A y = 1, so x0 = mean(b) 1."""
    n = 37
    b = np.random.default_rng(4).standard_normal(n)
    x0, a = O.initial_solution(np.eye(n), b)
    assert a == pytest.approx(b.mean(), rel=1e-14)
    np.testing.assert_allclose(x0, np.full(n, b.mean()), rtol=1e-13)


def test_initial_solution_remark_properties():
    """The remark after Algorithm 2: x0 in R(A^T) and RRN(x0) <= 1; from its
    proof, RRN(x0)^2 = 1 - <b, A y>^2 / (||b||^2 ||A y||^2) and the residual is
    orthogonal to A y."""
    rng = np.random.default_rng(9)
    A = rng.standard_normal((40, 90)) + 0.3      # wide: a null space exists
    b = rng.standard_normal(40)
    x0, a = O.initial_solution(A, b)
    r = b - A @ x0
    rrn = np.linalg.norm(r) / np.linalg.norm(b)
    assert rrn <= 1.0
    bt = A @ A.sum(axis=0)
    cos2 = (b @ bt) ** 2 / ((b @ b) * (bt @ bt))
    assert rrn ** 2 == pytest.approx(1.0 - cos2, rel=1e-10)
    assert abs(r @ bt) <= 1e-10 * np.linalg.norm(r) * np.linalg.norm(bt)
    coef = np.linalg.lstsq(A.T, x0, rcond=None)[0]          # x0 = A^T coef exactly?
    assert np.linalg.norm(A.T @ coef - x0) <= 1e-12 * np.linalg.norm(x0)


def test_initial_solution_degenerate_row_sum():
    """Rows that sum to zero give y = 0 and A y = 0: the coefficient is 0."""
    rng = np.random.default_rng(2)
    B = rng.integers(-9, 10, size=(10, 6)).astype(np.float64)   # exact sums
    A = np.vstack([B, -B])
    x0, a = O.initial_solution(A, rng.standard_normal(20))
    assert a == 0.0 and not np.any(x0)


def test_initial_solution_csr_matches_dense():
    s = csr_system(300, 5, cfg=5)
    x0c, ac = O.initial_solution(s, s["b"])
    D = O.Matrix(s).dense()
    x0d, ad = O.initial_solution(D, s["b"])
    assert ac == pytest.approx(ad, rel=1e-12)
    np.testing.assert_allclose(x0c, x0d, rtol=1e-12, atol=1e-300)


# ------------------------------------------- Algorithm 3 (flexible AB-GMRES)

def test_fabgmres_least_squares_property():
    """x_k = x0 + Z y with y minimising ||r0 - A Z y|| over the returned
    preconditioned directions, the rotated residual |g_{k+1}| equals the true
    ||b - A x_k||, and GMRES residuals never increase."""
    s = dense_svd_system(300, 120, 1e3, cfg=61)
    A, b = s["A"], s["b"]
    out = O.fabgmres(A, 20, 1e-3, b, seed=2, tol=1e-14, max_outer=12, inner_iters=3, eta=1e-6,
                     want_basis=True)
    k = out["outer"]
    assert k == 12
    Z = out["Z"]
    y = np.linalg.lstsq(A @ Z, b, rcond=None)[0]
    best = np.linalg.norm(b - A @ (Z @ y))
    got = np.linalg.norm(b - A @ out["x"])
    assert got == pytest.approx(best, rel=1e-8)
    assert out["res_hist"][-1] * np.linalg.norm(b) == pytest.approx(got, rel=1e-7)
    assert np.all(np.diff(out["res_hist"]) <= 1e-12)
    H = out["H"]
    assert np.all(np.abs(np.tril(H, -2)) == 0.0) and np.all(np.diag(H, -1) >= 0.0)


def test_fabgmres_row_space():
    """The remark after Algorithm 3: from x0 = 0 (and inner z0 = 0) the result
    lies in the row space of A."""
    s = dense_svd_system(60, 200, 1e2, cfg=62, rowspace=True)
    A = s["A"]
    out = O.fabgmres(A, 10, 1e-4, s["b"], seed=4, tol=1e-12, max_outer=8, inner_iters=2, eta=1e-8)
    x = out["x"]
    null = x - A.T @ np.linalg.solve(A @ A.T, A @ x)
    assert np.linalg.norm(null) <= 1e-10 * np.linalg.norm(x)


def test_fabgmres_exact_inner_solve_one_step():
    """One block of all rows: the inner ROR-BK step is the regularised
    pseudo-inverse A^T (A A^T + mu I)^{-1} v, so A z = v up to mu and the
    outer residual after one step is of the order of mu."""
    rng = np.random.default_rng(63)
    A = rng.standard_normal((40, 90))
    b = rng.standard_normal(40)
    mu = 1e-9
    out = O.fabgmres(A, 40, mu, b, seed=0, tol=1e-30, max_outer=1, inner_iters=1, eta=0.0)
    z = A.T @ np.linalg.solve(A @ A.T + mu * np.eye(40), b / np.linalg.norm(b))
    scale = np.linalg.norm(b) / np.linalg.norm(A @ z) ** 2 * (b @ (A @ z)) / np.linalg.norm(b)
    np.testing.assert_allclose(out["x"], scale * z, rtol=1e-8)
    assert out["res_hist"][0] < 1e-6
