"""The C ABI boundary, checked on the CPU: the built library loads and exports
every function include/rorbk.h declares, the binding's constants and struct
layouts agree with the header, and the product path refuses to run without
the HIP library (there is no CPU fallback).  No call here touches a device."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rorbk.h")


def _header():
    with open(HEADER) as f:
        return f.read()


def _declared_functions():
    src = re.sub(r"/\*.*?\*/", "", _header(), flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(ror_bk_\w+)\s*\(", src, re.M)))


def _defines():
    return {k: int(v) for k, v in
            re.findall(r"^#define\s+(RORBK_\w+)\s+(\d+)u?\b", _header(), re.M)}


def test_header_declares_the_binding_exports():
    from paper_2510_02156_amd import binding
    assert _declared_functions() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2510_02156_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("librorbk.so not built (run __graft_entry__.build())")
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = [f for f in _declared_functions() if f not in exported]
    assert not missing, missing
    # and the dynamic loader resolves each of them
    L = C.CDLL(binding.LIB_PATH)
    for f in _declared_functions():
        assert getattr(L, f) is not None


def test_error_strings_cover_every_status():
    from paper_2510_02156_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("librorbk.so not built")
    L = binding.lib()
    codes = {k: v for k, v in _defines().items() if k.startswith("RORBK_OK") or
             k.startswith("RORBK_ERR_")}
    texts = {L.ror_bk_error_string(v).decode() for v in codes.values()}
    assert len(texts) == len(codes)          # one distinct message per status
    assert L.ror_bk_error_string(999).decode()  # unknown codes still get text


def test_binding_constants_match_header():
    from paper_2510_02156_amd import binding
    d = _defines()
    for name, val in d.items():
        if name in ("RORBK_H",):
            continue
        assert getattr(binding, name) == val, name


def test_struct_layouts_match_header():
    from paper_2510_02156_amd import binding
    # rorbk_matrix: 2 int32, 3 int64, 3 pointers, int64, pointer (x86-64 / LP64)
    assert C.sizeof(binding.rorbk_matrix) == 8 + 3 * 8 + 3 * 8 + 8 + 8
    assert binding.rorbk_matrix.values.offset == 32
    assert binding.rorbk_matrix.values_f64.offset == 64
    # rorbk_info: int64, double, 2 int32, 3 doubles
    assert C.sizeof(binding.rorbk_info) == 48
    assert binding.rorbk_info.t_solve_s.offset == 24
    assert binding.rorbk_info.t_setup_s.offset == 32
    assert binding.rorbk_info.rrn_test.offset == 40
    # and the header lists the same fields in the same order
    body = re.search(r"typedef struct rorbk_info \{(.*?)\} rorbk_info;", _header(), re.S).group(1)
    names = re.findall(r"^\s*\w+\s+(\w+);", re.sub(r"/\*.*?\*/", "", body, flags=re.S), re.M)
    assert names == [f[0] for f in binding.rorbk_info._fields_]


def test_partition_entry_point_matches_oracle():
    """ror_bk_partition (host, no handle, no device) against the oracle's
    partition for every block size 1..m on several m, bit for bit; the
    argument checks refuse the degenerate requests."""
    from paper_2510_02156_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("librorbk.so not built")
    import numpy as np

    import oracle as O
    for m in (1, 2, 3, 7, 64, 100, 257, 1000, 2001):
        for br in range(1, m + 1):
            got = binding.ror_bk_partition(m, br)
            ref = O.partition(m, br)
            assert got.dtype == np.int64 and np.array_equal(got, ref), (m, br)
    # the full sizes of the dense, tall, sparse, wide and differentiation workloads
    for m, br in ((2000, 20), (100000, 64), (200000, 128), (2000, 32), (20000, 50)):
        assert np.array_equal(binding.ror_bk_partition(m, br), O.partition(m, br))
    L = binding.lib()
    k = C.c_int64(-1)
    for m, br in ((0, 1), (5, 0), (5, 6), (-3, 1)):
        assert L.ror_bk_partition(m, br, None, C.byref(k)) == binding.RORBK_ERR_INVALID_ARG
    assert L.ror_bk_partition(10, 3, None, None) == binding.RORBK_ERR_INVALID_ARG
    assert L.ror_bk_partition(10, 3, None, C.byref(k)) == binding.RORBK_OK and k.value == 3


def test_every_declaration_cites_the_paper_or_says_why_not():
    """Each entry point's comment names the passage of the paper it implements
    (an algorithm, section or lemma), or states that it is not a step of the
    method."""
    text = _header()
    for name in _declared_functions():
        m = re.search(r"/\*((?:(?!\*/).)*?)\*/\s*(?:int|const char \*)\s*" + name + r"\s*\(",
                      text, re.S)
        assert m, f"{name} has no comment right above it"
        doc = m.group(1)
        assert re.search(r"Algorithm \d|Section \d|Sec\. \d|Lemma \d|not in the paper|"
                         r"paper defines no|not a step of the method|callers that cannot", doc), name


def test_block_size_limits_refused_before_any_device_call():
    """Blocks above the supported sizes (2048 rows dense, 161 rows CSR) are
    refused with RORBK_ERR_UNSUPPORTED by the argument checks, which run
    before the library touches a device (the pointers are never read)."""
    from paper_2510_02156_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("librorbk.so not built")
    L = binding.lib()
    fake = C.c_void_p(0x1000)
    h = C.c_void_p()
    for fmt, m, br in [(binding.RORBK_DENSE, 2 * 2049, 2049),
                       (binding.RORBK_CSR, 2 * 162, 162)]:
        A = binding.rorbk_matrix(format=fmt, dtype=binding.RORBK_F64, m=m, n=m, ld=m,
                                 values=fake, rowptr=fake, colidx=fake, nnz=m,
                                 values_f64=None)
        rc = L.ror_bk_setup(C.byref(A), C.c_int64(br), C.c_double(1e-3), None, C.byref(h))
        assert rc == binding.RORBK_ERR_UNSUPPORTED
        assert not h.value
        assert b"exceed" in L.ror_bk_last_error_message()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2510_02156_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "librorbk.so"))
    with pytest.raises(ImportError):
        binding.lib()


def test_product_path_does_not_reach_the_oracle():
    """Nothing under the package imports, links or reads the oracle."""
    pkg = os.path.join(ROOT, "paper_2510_02156_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if not fn.endswith((".py", ".hip", ".h", ".cpp", ".c")):
                continue
            with open(os.path.join(dirpath, fn)) as f:
                text = f.read()
            assert "oracle" not in text.lower(), os.path.join(dirpath, fn)


def test_noalloc_residual_refuses_oversized_problems_before_any_device_call():
    """ror_bk_residual_noalloc checks its arguments and the size of its static
    scratch on the host: a problem whose partial products exceed the array
    (RORBK_NOALLOC_SCRATCH_BYTES) is refused with RORBK_ERR_UNSUPPORTED, and
    bad arguments with RORBK_ERR_INVALID_ARG, before anything reaches a
    device (the pointers below are never dereferenced)."""
    from paper_2510_02156_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("librorbk.so not built")
    L = binding.lib()
    fake = C.c_void_p(0x1000)
    cap = binding.RORBK_NOALLOC_SCRATCH_BYTES
    m = cap // 8 + 1          # one segment of partial products alone exceeds the array
    A = binding.rorbk_matrix(format=binding.RORBK_DENSE, dtype=binding.RORBK_F64, m=m, n=100,
                             ld=100, values=fake, rowptr=None, colidx=None, nnz=0,
                             values_f64=None)
    rc = L.ror_bk_residual_noalloc(C.byref(A), 64, fake, fake, fake, None, None, 0, None)
    assert rc == binding.RORBK_ERR_UNSUPPORTED
    assert b"scratch" in L.ror_bk_last_error_message()
    # several column segments multiply the need: 3 segments of 1e6 rows
    A.m, A.n, A.ld = 1000000, 5000, 5000
    assert L.ror_bk_residual_noalloc(C.byref(A), 64, fake, fake, fake, None, None, 0,
                                     None) == binding.RORBK_ERR_UNSUPPORTED
    # argument errors
    A.m, A.n, A.ld = 1000, 100, 100
    assert L.ror_bk_residual_noalloc(C.byref(A), 0, fake, fake, fake, None, None, 0,
                                     None) == binding.RORBK_ERR_INVALID_ARG
    assert L.ror_bk_residual_noalloc(C.byref(A), 10, None, fake, fake, None, None, 0,
                                     None) == binding.RORBK_ERR_INVALID_ARG
    assert L.ror_bk_residual_noalloc(C.byref(A), 10, fake, fake, fake, None, None, 1,
                                     None) == binding.RORBK_ERR_INVALID_ARG   # float vs F64
    A.dtype = binding.RORBK_F32
    assert L.ror_bk_residual_noalloc(C.byref(A), 10, fake, fake, fake, None, None, 0,
                                     None) == binding.RORBK_ERR_INVALID_ARG   # no FP64 master
    A.dtype = binding.RORBK_F64
    A.m = 10000
    assert L.ror_bk_residual_noalloc(C.byref(A), 2049, fake, fake, fake, None, None, 0,
                                     None) == binding.RORBK_ERR_UNSUPPORTED   # block rows
