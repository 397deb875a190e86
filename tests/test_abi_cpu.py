"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects malformed input on the host side with the documented
status codes (include/sparsespec.h)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sparsespec.h")


@pytest.fixture(scope="module")
def ss():
    from paper_2302_00752_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_2302_00752_amd import sparsespec
    return sparsespec


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ss_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("ss_build_stamp", "ss_build_stamp_batch", "ss_build_op", "ss_apply", "ss_solve",
                 "ss_solve_op", "ss_stamp_lookup", "ss_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(ss):
    lib = C.CDLL(ss.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(ss.EXPORTED) <= set(declared_symbols())
    assert "gfx950" in ss.version()


def _build(ss, d, a, f, level=1):
    a = np.ascontiguousarray(a, dtype=np.int16)
    f = np.ascontiguousarray(f, dtype=np.int16)
    h = C.c_void_p()
    st = ss._lib.ss_build_stamp(d, len(a), ss._ptr(a, C.c_int16), len(f), ss._ptr(f, C.c_int16), level,
                                None, C.byref(h))
    return st, ss._lib.ss_last_error().decode()


def test_stamp_argument_errors(ss):
    assert _build(ss, 0, [[0]], [[1]])[0] == ss.SS_EINVAL                       # d out of range
    st, msg = _build(ss, 2, [[1, 0]], [[1, 1]])                                 # 0 not in supp(a)
    assert st == ss.SS_EINVAL and "supp(a)" in msg
    assert _build(ss, 2, [[0, 0], [1, 0], [1, 0]], [[1, 1]])[0] == ss.SS_EINVAL  # duplicate w
    assert _build(ss, 2, [[0, 0]], [[1, 1], [1, 1]])[0] == ss.SS_EINVAL          # duplicate f
    assert _build(ss, 2, [[0, 0]], [[1, 1]], level=-1)[0] == ss.SS_EINVAL        # level
    assert _build(ss, 2, [[0, 0], [-32768, 0]], [[1, 1]])[0] == ss.SS_ERANGE     # -w not in int16
    many = [[0, 0]] + [[i, 1] for i in range(1, 65)]                             # 129 after closure
    assert _build(ss, 2, many, [[1, 1]])[0] == ss.SS_ERANGE


def _solve(ss, d, af, ah, ff, fh, level=1):
    af = np.ascontiguousarray(af, dtype=np.int16).reshape(-1, d)
    ff = np.ascontiguousarray(ff, dtype=np.int16).reshape(-1, d)
    ah = np.ascontiguousarray(np.asarray(ah, dtype=np.complex128)).view(np.float64)
    fh = np.ascontiguousarray(np.asarray(fh, dtype=np.complex128)).view(np.float64)
    n = C.c_int64()
    st = ss._lib.ss_solve(d, len(af), ss._ptr(af, C.c_int16), ss._ptr(ah, C.c_double), len(ff),
                          ss._ptr(ff, C.c_int16), ss._ptr(fh, C.c_double), level, 1e-10, 0, 100, 0, None, 0,
                          C.byref(n), None, None, None)
    return st, ss._lib.ss_last_error().decode()


def test_solve_argument_errors(ss):
    a0 = [[0, 0], [1, 0], [-1, 0]]
    # coefficients at w and -w not conjugate: a would not be real
    st, msg = _solve(ss, 2, a0, [1.0, 0.1 + 0.1j, 0.1 + 0.1j], [[0, 1]], [1.0])
    assert st == ss.SS_EINVAL and "conjugate" in msg
    # a_0 must be real and positive
    assert _solve(ss, 2, a0, [-1.0, 0.1, 0.1], [[0, 1]], [1.0])[0] == ss.SS_EINVAL
    assert _solve(ss, 2, a0, [1.0 + 0.5j, 0.1, 0.1], [[0, 1]], [1.0])[0] == ss.SS_EINVAL
    # mean-zero forcing (Prop. ExistenceUniquenessStability)
    st, msg = _solve(ss, 2, a0, [1.0, 0.1, 0.1], [[0, 0], [0, 1]], [1.0, 1.0])
    assert st == ss.SS_EINVAL and "f_0" in msg
    # no nonzero forcing coefficient
    assert _solve(ss, 2, a0, [1.0, 0.1, 0.1], [[0, 1]], [0.0])[0] == ss.SS_EINVAL
    # non-finite input
    assert _solve(ss, 2, a0, [1.0, np.nan, 0.1], [[0, 1]], [1.0])[0] == ss.SS_EINVAL


def test_binding_rejects_out_of_range_keys(ss):
    with pytest.raises(ss.SparseSpecError):
        ss._i16(np.array([[40000, 0]]))


def test_memory_stats_without_a_device(ss):
    # the allocator's counters need no device: nothing allocated yet in a CPU-only process
    m = ss.memory_stats()
    assert m == {"live_bytes": 0, "cached_bytes": 0, "driver_allocs": 0}
    assert ss._lib.ss_memory_stats(None, None, None) == ss.SS_EINVAL
