"""The allocation-free residual entry point (ror_bk_residual_noalloc) against
the handle-based ror_bk_residual, through the C ABI: the same kernels run on
the same inputs, so r and the per-block norms must agree bit for bit and the
RRN to rounding of its last division.  Two calls in a row on each case, the
second on a smaller problem, check that nothing of the first call's scratch
contents leaks into the second (the static array keeps the last call's
contents)."""
import numpy as np
import pytest

from workloads import csr_system, dense_svd_system

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2510_02156_amd as P  # noqa: E402
from paper_2510_02156_amd import binding  # noqa: E402
from tests.gpu_util import bf16_tensor, dev  # noqa: E402


def _dense_case(m, n, storage, br, vec, seed):
    s = dense_svd_system(m, n, 1e3, cfg=seed)
    A64 = dev(s["A"])
    if storage == "f64":
        At = A64
    elif storage == "f32":
        At = A64.float()
    else:
        At = bf16_tensor(s["A"])
    rng = np.random.default_rng(seed)
    vt = torch.float32 if vec == "f32" else torch.float64
    b = dev(s["b"], vt)
    x = dev(rng.standard_normal(n), vt)
    desc = binding.matrix_descriptor(At, A64=A64)
    sol = P.Solver(At, br, 1e-3, A64=A64)
    return desc, sol, b, x, (At, A64)


def _csr_case(m, br, seed):
    w = csr_system(m, 12, cfg=seed)
    rowptr = torch.from_numpy(w["rowptr"]).to("cuda:0")
    colidx = torch.from_numpy(w["colidx"]).to("cuda:0")
    vals = torch.from_numpy(w["val"]).to("cuda:0")
    rng = np.random.default_rng(seed)
    b = dev(w["b"])
    x = dev(rng.standard_normal(m))
    desc = binding.matrix_descriptor(rowptr=rowptr, colidx=colidx, values=vals, shape=(m, m))
    sol = P.Solver(None, br, 1e-4, rowptr=rowptr, colidx=colidx, values=vals, shape=(m, m))
    return desc, sol, b, x, (rowptr, colidx, vals)


def _compare(desc, sol, b, x, br, label):
    k = sol.k
    m = sol.m
    r0, bn0, rrn0 = sol.residual(b, x, use_f64_master=(b.dtype == torch.float64))
    r = torch.full((m,), float("nan"), dtype=b.dtype, device="cuda:0")
    bn = torch.full((k,), float("nan"), dtype=torch.float64, device="cuda:0")
    rrn = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda:0")
    binding.ror_bk_residual_noalloc(desc, br, b, x, r, bn, rrn)
    torch.cuda.synchronize()
    assert torch.equal(r, r0), label
    assert torch.equal(bn, bn0), label
    got = float(rrn.item())
    print(f"{label}: rrn {got:.6e} (handle entry point {rrn0:.6e})", flush=True)
    assert got == pytest.approx(rrn0, rel=1e-15, abs=0.0)
    # without the block norms (kept in the static array instead)
    r2 = torch.zeros_like(r)
    rrn2 = torch.zeros_like(rrn)
    binding.ror_bk_residual_noalloc(desc, br, b, x, r2, None, rrn2)
    torch.cuda.synchronize()
    assert torch.equal(r2, r0) and float(rrn2.item()) == got


@pytest.mark.parametrize("storage,vec", [("f64", "f64"), ("f32", "f32"), ("bf16", "f32"),
                                         ("f32", "f64")])
def test_noalloc_residual_matches_entry_point_dense(storage, vec):
    # first call: 3 column segments and ragged blocks; second: a smaller one
    for (m, n, br, seed) in ((5003, 4500, 64, 61), (777, 300, 20, 62)):
        print(f"noalloc dense {storage}/{vec} m={m} n={n} br={br}", flush=True)
        desc, sol, b, x, keep = _dense_case(m, n, storage, br, vec, seed)
        _compare(desc, sol, b, x, br, f"dense {storage}/{vec} {m}x{n}")
        sol.close()


def test_noalloc_residual_matches_entry_point_csr():
    for (m, br, seed) in ((20011, 128, 63), (3001, 32, 64)):
        print(f"noalloc csr m={m} br={br}", flush=True)
        desc, sol, b, x, keep = _csr_case(m, br, seed)
        _compare(desc, sol, b, x, br, f"csr {m}")
        sol.close()


def test_noalloc_residual_full_tall_size():
    """The tall workload's shape (100000 x 2000, blocks of 64 rows) in FP32
    storage, the configuration of the benchmark's residual pass."""
    s = dense_svd_system(100000, 2000, 1e8, cfg=65)
    A64 = dev(s["A"])
    A32 = A64.float()
    rng = np.random.default_rng(65)
    b = dev(s["b"], torch.float32)
    x = dev(rng.standard_normal(2000), torch.float32)
    print("noalloc full tall FP32", flush=True)
    desc = binding.matrix_descriptor(A32, A64=A64)
    sol = P.Solver(A32, 64, 1e-4, A64=A64)
    _compare(desc, sol, b, x, 64, "tall 100000x2000 f32")
    sol.close()
