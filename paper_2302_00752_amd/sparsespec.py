"""Python binding of ``libsparsespec`` (ctypes; argument marshalling only).

Every computation happens in the HIP library.  PyTorch provides device
memory (tensors' ``data_ptr()``) and the current HIP stream.  If the built
library is missing, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsparsespec.so")

SS_OK, SS_EINVAL, SS_ENOMEM, SS_ERANGE, SS_ENOTPD, SS_ENOCONV, SS_EBREAKDOWN, SS_EDEVICE = range(8)
SS_FP64, SS_FP32_REFINE = 0, 1
SS_SKIP_L1_CHECK = 1
SS_EXACT_LOOKUP = 2
STATUS_NAMES = {0: "SS_OK", 1: "SS_EINVAL", 2: "SS_ENOMEM", 3: "SS_ERANGE", 4: "SS_ENOTPD",
                5: "SS_ENOCONV", 6: "SS_EBREAKDOWN", 7: "SS_EDEVICE"}
PRECISION = {"fp64": SS_FP64, "fp32_refine": SS_FP32_REFINE, SS_FP64: SS_FP64, SS_FP32_REFINE: SS_FP32_REFINE}

EXPORTED = ["ss_build_stamp_batch", "ss_build_stamp", "ss_stamp_size", "ss_stamp_keys", "ss_stamp_lookup",
            "ss_stamp_lookup_batch", "ss_stamp_forcing",
            "ss_free_stamp", "ss_build_op", "ss_op_info", "ss_op_csr", "ss_op_exec_map", "ss_apply",
            "ss_solve_op", "ss_free_op", "ss_solve", "ss_last_error", "ss_version", "ss_op_bytes",
            "ss_engine_create", "ss_engine_submit", "ss_engine_step", "ss_engine_poll", "ss_engine_usage",
            "ss_engine_free", "ss_solve_batch", "ss_batch_size", "ss_batch_solution", "ss_free_batch",
            "ss_proxy_error", "ss_solve_direct", "ss_op_class_sizes", "ss_build_adr", "ss_adr_apply",
            "ss_adr_solve", "ss_free_adr", "ss_lattice_modulus", "ss_stamp_lattice", "ss_solve_op_noalloc",
            "ss_memory_stats"]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_steps", C.c_int32), ("rel_residual", C.c_double),
                ("n", C.c_int64), ("nnz", C.c_int64), ("n_components", C.c_int32), ("status", C.c_int32),
                ("t_build_ms", C.c_double), ("t_solve_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class DirectInfo(C.Structure):
    _fields_ = [("factor_ms", C.c_double), ("tiles", C.c_int64), ("chunks", C.c_int32), ("refine_steps", C.c_int32),
                ("rel_residual", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SparseSpecError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2302_00752_amd.build`")
    lib = C.CDLL(path)
    P = C.c_void_p
    i32, i64, u32, dbl = C.c_int32, C.c_int64, C.c_uint32, C.c_double
    pi32, pi64, pi16, pu8, pd = (C.POINTER(i32), C.POINTER(i64), C.POINTER(C.c_int16),
                                 C.POINTER(C.c_uint8), C.POINTER(dbl))
    sig = {
        "ss_build_stamp_batch": [i32, i32, pi32, pi16, pi32, pi16, pi32, P, C.POINTER(P)],
        "ss_build_stamp": [i32, i32, pi16, i32, pi16, i32, P, C.POINTER(P)],
        "ss_stamp_size": [P, pi64, pi32, pi64],
        "ss_stamp_keys": [P, pi16, pu8],
        "ss_stamp_lookup": [P, i32, i64, pi16, pi64],
        "ss_stamp_lookup_batch": [P, i64, pi32, pi16, pi64],
        "ss_stamp_forcing": [P, pd, P, P],
        "ss_lattice_modulus": [i64, i64, dbl, pi64],
        "ss_stamp_lattice": [P, pi64, i64, P, pi32, P],
        "ss_build_op": [P, pi32, pi16, pd, u32, P, C.POINTER(P)],
        "ss_op_info": [P, pi64, pi64, pi64, pi64],
        "ss_op_csr": [P, pi64, pi32, pi32, pi32],
        "ss_op_exec_map": [P, pi64],
        "ss_apply": [P, i32, P, P, P],
        "ss_solve_op": [P, P, P, dbl, i32, i32, P, C.POINTER(SolveInfo)],
        "ss_solve_op_noalloc": [P, P, P, dbl, i32, i32, P, C.POINTER(SolveInfo)],
        "ss_solve": [i32, i32, pi16, pd, i32, pi16, pd, i32, dbl, i32, i32, u32, pd, i64, pi64, pd, pi16,
                     C.POINTER(SolveInfo)],
        "ss_op_bytes": [P, pi64],
        "ss_memory_stats": [pi64, pi64, pi64],
        "ss_engine_create": [i64, i32, P, C.POINTER(P)],
        "ss_engine_submit": [P, P, P, P, dbl, i32, i32, i64],
        "ss_engine_step": [P, i32, pi32],
        "ss_engine_poll": [P, i32, pi64, pi32, C.POINTER(SolveInfo), pi32],
        "ss_engine_usage": [P, pi32, pi64],
        "ss_solve_batch": [i32, i32, pi32, pi16, pd, pi32, pi16, pd, pi32, dbl, i32, i32, u32, i32, C.POINTER(P),
                           C.POINTER(SolveInfo)],
        "ss_batch_size": [P, pi64, pi64],
        "ss_batch_solution": [P, P, P],
        "ss_proxy_error": [P, P, P, i64, pd, pd, P],
        "ss_solve_direct": [P, P, P, i32, dbl, P, C.POINTER(DirectInfo)],
        "ss_op_class_sizes": [P, i64, pi64, pi64],
        "ss_build_adr": [P, P, pi32, pi16, pd, pi32, pi16, pd, P, C.POINTER(P)],
        "ss_adr_apply": [P, P, P, P],
        "ss_adr_solve": [P, P, P, dbl, i32, P, C.POINTER(SolveInfo)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.ss_free_stamp.argtypes = [P]
    lib.ss_free_stamp.restype = None
    lib.ss_free_op.argtypes = [P]
    lib.ss_free_op.restype = None
    lib.ss_engine_free.argtypes = [P]
    lib.ss_engine_free.restype = None
    lib.ss_free_adr.argtypes = [P]
    lib.ss_free_adr.restype = None
    lib.ss_free_batch.argtypes = [P]
    lib.ss_free_batch.restype = None
    lib.ss_last_error.restype = C.c_char_p
    lib.ss_version.restype = C.c_char_p
    return lib


_lib = load()


def _check(status: int):
    if status != SS_OK:
        raise SparseSpecError(status, _lib.ss_last_error().decode())


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _i16(a) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype != np.int16:
        if a.size and (a.min() < -32768 or a.max() > 32767):
            raise SparseSpecError(SS_ERANGE, "frequency coordinate outside int16")
        a = a.astype(np.int16)
    return a


def _c128(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    return a.view(np.float64)


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


class Batch:
    """Problems of one dimension packed once into the flat host arrays the C ABI
    takes (objects with ``d, a_freqs, f_freqs, level`` and, where present,
    ``a_hat, f_hat``).  Builds accept a ``Batch`` or the list of problems."""

    def __init__(self, problems: Sequence):
        d = int(problems[0].d)
        if any(int(p.d) != d for p in problems):
            raise SparseSpecError(SS_EINVAL, "a batch must share the dimension d")
        self.d = d
        self.n_prob = len(problems)
        self.n_a = np.array([len(p.a_freqs) for p in problems], dtype=np.int32)
        self.n_f = np.array([len(p.f_freqs) for p in problems], dtype=np.int32)
        self.level = np.array([int(p.level) for p in problems], dtype=np.int32)
        self.a_freqs = _i16(np.concatenate([np.asarray(p.a_freqs).reshape(-1, d) for p in problems]))
        self.f_freqs = _i16(np.concatenate([np.asarray(p.f_freqs).reshape(-1, d) for p in problems]))
        has_a = all(getattr(p, "a_hat", None) is not None for p in problems)
        has_f = all(getattr(p, "f_hat", None) is not None for p in problems)
        self.a_hat = _c128(np.concatenate([np.asarray(p.a_hat) for p in problems])) if has_a else None
        self.f_hat = _c128(np.concatenate([np.asarray(p.f_hat) for p in problems])) if has_f else None


def _batch(problems) -> Batch:
    return problems if isinstance(problems, Batch) else Batch(problems)


class Stamp:
    """Stamping sets S^N of a batch of problems of one dimension (device-resident)."""

    def __init__(self, handle, d: int, n_f: int = -1):
        self._h = handle
        self.d = d
        self.n_f = n_f           # forcing frequencies given to the build
        n = C.c_int64()
        npb = C.c_int32()
        _check(_lib.ss_stamp_size(self._h, C.byref(n), C.byref(npb), None))
        self.n_total = n.value
        self.n_prob = npb.value
        off = np.zeros(self.n_prob + 1, dtype=np.int64)
        _check(_lib.ss_stamp_size(self._h, None, None, _ptr(off, C.c_int64)))
        self.offsets = off

    @classmethod
    def build(cls, problems, stream=None) -> "Stamp":
        """Build from a ``Batch`` or a list of problems of one dimension."""
        b = _batch(problems)
        h = C.c_void_p()
        _check(_lib.ss_build_stamp_batch(b.n_prob, b.d, _ptr(b.n_a, C.c_int32), _ptr(b.a_freqs, C.c_int16),
                                         _ptr(b.n_f, C.c_int32), _ptr(b.f_freqs, C.c_int16),
                                         _ptr(b.level, C.c_int32), C.c_void_p(_stream(stream)), C.byref(h)))
        return cls(h, b.d, int(b.n_f.sum()))

    def keys(self):
        k = np.zeros((self.n_total, self.d), dtype=np.int16)
        lev = np.zeros(self.n_total, dtype=np.uint8)
        _check(_lib.ss_stamp_keys(self._h, _ptr(k, C.c_int16), _ptr(lev, C.c_uint8)))
        return k, lev

    def lookup(self, prob: int, q) -> np.ndarray:
        q = _i16(np.asarray(q).reshape(-1, self.d))
        out = np.zeros(len(q), dtype=np.int64)
        _check(_lib.ss_stamp_lookup(self._h, int(prob), len(q), _ptr(q, C.c_int16), _ptr(out, C.c_int64)))
        return out

    def lookup_batch(self, prob, q) -> np.ndarray:
        """Global canonical slots of keys ``q`` of problems ``prob`` (-1 if absent)."""
        q = _i16(np.asarray(q).reshape(-1, self.d))
        prob = np.ascontiguousarray(prob, dtype=np.int32)
        out = np.zeros(len(q), dtype=np.int64)
        _check(_lib.ss_stamp_lookup_batch(self._h, len(q), _ptr(prob, C.c_int32), _ptr(q, C.c_int16),
                                          _ptr(out, C.c_int64)))
        return out

    def forcing_vector(self, problems, device=None, stream=None):
        """f in canonical slot order (complex128 tensor on ``device``): each problem's
        f_hat at the slots of its forcing frequencies (the batch the stamp was built from)."""
        import torch
        vals = problems.f_hat if isinstance(problems, Batch) else \
            _c128(np.concatenate([np.asarray(p.f_hat) for p in problems]))
        if vals is None or len(vals) != 2 * self.n_f:
            raise SparseSpecError(SS_EINVAL, "one f_hat coefficient per forcing frequency of the build is needed")
        f = torch.empty(self.n_total, dtype=torch.complex128, device=device or "cuda")
        _check(_lib.ss_stamp_forcing(self._h, _ptr(vals, C.c_double), C.c_void_p(f.data_ptr()),
                                     C.c_void_p(_stream(stream))))
        return f

    def lattice(self, z, M, values=True, stream=None):
        """Rank-1 lattice Lambda(z, M) on every problem's set (Sec. 8, Lemma
        RandomRank1Lattice): (reconstructing, values) with reconstructing a bool array per
        problem and values the int64 tensor of k . z mod M per key in canonical order (None
        when ``values`` is false)."""
        import torch
        z = np.ascontiguousarray(np.asarray(z, dtype=np.int64))
        if z.shape != (self.d,):
            raise SparseSpecError(SS_EINVAL, "z needs one entry per dimension")
        ok = np.zeros(self.n_prob, dtype=np.int32)
        vals = torch.empty(self.n_total, dtype=torch.int64, device="cuda") if values else None
        _check(_lib.ss_stamp_lattice(self._h, _ptr(z, C.c_int64), int(M),
                                     C.c_void_p(vals.data_ptr() if values else 0), _ptr(ok, C.c_int32),
                                     C.c_void_p(_stream(stream))))
        return ok.astype(bool), vals

    def close(self):
        if self._h:
            _lib.ss_free_stamp(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """Truncated Galerkin operators L_N of a stamped batch (device-resident)."""

    def __init__(self, handle, stamp: Stamp):
        self._h = handle
        self.n_prob = stamp.n_prob
        self.offsets = stamp.offsets.copy()
        vals = [C.c_int64() for _ in range(4)]
        _check(_lib.ss_op_info(self._h, *[C.byref(v) for v in vals]))
        self.n_total, self.n_exec, self.nnz, self.n_components = [v.value for v in vals]

    @classmethod
    def build(cls, stamp: Stamp, problems, flags: int = 0, stream=None) -> "Operator":
        b = _batch(problems)
        if b.a_hat is None:
            raise SparseSpecError(SS_EINVAL, "the operator needs a_hat of every problem")
        h = C.c_void_p()
        _check(_lib.ss_build_op(stamp._h, _ptr(b.n_a, C.c_int32), _ptr(b.a_freqs, C.c_int16),
                                _ptr(b.a_hat, C.c_double), int(flags), C.c_void_p(_stream(stream)), C.byref(h)))
        return cls(h, stamp)

    def csr(self):
        rp = np.zeros(self.n_total + 1, dtype=np.int64)
        cols = np.zeros(max(self.nnz, 1), dtype=np.int32)
        js = np.zeros(max(self.nnz, 1), dtype=np.int32)
        comp = np.zeros(self.n_total, dtype=np.int32)
        _check(_lib.ss_op_csr(self._h, _ptr(rp, C.c_int64), _ptr(cols, C.c_int32), _ptr(js, C.c_int32),
                              _ptr(comp, C.c_int32)))
        return rp, cols[:self.nnz], js[:self.nnz], comp

    def exec_map(self) -> np.ndarray:
        m = np.zeros(self.n_exec, dtype=np.int64)
        _check(_lib.ss_op_exec_map(self._h, _ptr(m, C.c_int64)))
        return m

    def apply(self, x, y, precision="fp64", stream=None):
        """y = L_N x on device tensors in execution order (complex128 / complex64)."""
        _check(_lib.ss_apply(self._h, PRECISION[precision], C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                             C.c_void_p(_stream(stream))))

    def solve(self, f, u, tol: float, precision="fp64", max_iter: int = 1000, stream=None,
              raise_on_error: bool = True) -> List[dict]:
        """Solve L_N u = f in place (device complex128 tensors, canonical order)."""
        info = (SolveInfo * self.n_prob)()
        st = _lib.ss_solve_op(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), float(tol),
                              PRECISION[precision], int(max_iter), C.c_void_p(_stream(stream)), info)
        if raise_on_error:
            _check(st)
        return [i.as_dict() for i in info]

    def solve_noalloc(self, f, u, tol: float, precision="fp64", max_iter: int = 1000, stream=None,
                      raise_on_error: bool = True) -> List[dict]:
        """``solve`` without allocation (ss_solve_op_noalloc): operators whose classes have at
        most 2048 rows; the launch tables live in the library's fixed per-GPU array."""
        info = (SolveInfo * self.n_prob)()
        st = _lib.ss_solve_op_noalloc(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), float(tol),
                                      PRECISION[precision], int(max_iter), C.c_void_p(_stream(stream)), info)
        if raise_on_error:
            _check(st)
        return [i.as_dict() for i in info]

    def solve_direct(self, f, u, precision="fp64", tol: float = 0.0, stream=None) -> dict:
        """Dense direct solve of L_N u = f per connected class (device complex128, canonical order);
        ``tol > 0`` refines until every class's relative residual is below it."""
        info = DirectInfo()
        _check(_lib.ss_solve_direct(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()),
                                    PRECISION[precision], float(tol), C.c_void_p(_stream(stream)), C.byref(info)))
        return info.as_dict()

    def class_sizes(self) -> np.ndarray:
        """Rows of every connected class, in execution order."""
        n = C.c_int64()
        _check(_lib.ss_op_class_sizes(self._h, 0, None, C.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.int64)
        _check(_lib.ss_op_class_sizes(self._h, int(n.value), _ptr(out, C.c_int64), C.byref(n)))
        return out[:n.value]

    def device_bytes(self) -> int:
        b = C.c_int64()
        _check(_lib.ss_op_bytes(self._h, C.byref(b)))
        return b.value

    def close(self):
        if self._h:
            _lib.ss_free_op(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AdrOperator:
    """Advection-diffusion-reaction operators (Remark ADR) on a stamp and operator built on the
    union support (``problem.diffusion_on_union()``); the operator must outlive this object."""

    def __init__(self, handle, op: "Operator"):
        self._h = handle
        self.op = op
        self.n_prob = op.n_prob

    @classmethod
    def build(cls, stamp: Stamp, op: "Operator", problems, stream=None) -> "AdrOperator":
        d = stamp.d
        n_b = np.array([len(p.b_freqs) for p in problems], dtype=np.int32)
        n_c = np.array([len(p.c_freqs) for p in problems], dtype=np.int32)
        bf = _i16(np.concatenate([np.asarray(p.b_freqs).reshape(-1, d) for p in problems]))
        bh = _c128(np.concatenate([np.asarray(p.b_hat).reshape(-1, d) for p in problems]).ravel())
        cf = _i16(np.concatenate([np.asarray(p.c_freqs).reshape(-1, d) for p in problems]))
        ch = _c128(np.concatenate([np.asarray(p.c_hat) for p in problems]))
        h = C.c_void_p()
        _check(_lib.ss_build_adr(stamp._h, op._h, _ptr(n_b, C.c_int32), _ptr(bf, C.c_int16), _ptr(bh, C.c_double),
                                 _ptr(n_c, C.c_int32), _ptr(cf, C.c_int16), _ptr(ch, C.c_double),
                                 C.c_void_p(_stream(stream)), C.byref(h)))
        return cls(h, op)

    def apply(self, x, y, stream=None):
        """y = L x (device complex128, execution order)."""
        _check(_lib.ss_adr_apply(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                 C.c_void_p(_stream(stream))))

    def solve(self, f, u, tol: float, max_iter: int = 2000, stream=None, raise_on_error: bool = True) -> List[dict]:
        """Solve L u = f (device complex128, canonical order) by BiCGSTAB."""
        info = (SolveInfo * self.n_prob)()
        st = _lib.ss_adr_solve(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), float(tol),
                               int(max_iter), C.c_void_p(_stream(stream)), info)
        if raise_on_error:
            _check(st)
        return [i.as_dict() for i in info]

    def close(self):
        if self._h:
            _lib.ss_free_adr(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Engine:
    """Continuous-batching solver engine (see ss_engine_* in include/sparsespec.h)."""

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 0, stream=None):
        self._h = C.c_void_p()
        self._stream = _stream(stream)
        _check(_lib.ss_engine_create(int(hbm_budget_bytes), int(max_slots), C.c_void_p(self._stream),
                                     C.byref(self._h)))

    def submit(self, op: "Operator", f, u, tol: float, precision="fp64", max_iter: int = 1000,
               tag: int = 0) -> bool:
        """Admit op's problems; False (nothing admitted) if budget or slots are exhausted."""
        st = _lib.ss_engine_submit(self._h, op._h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()),
                                   float(tol), PRECISION[precision], int(max_iter), int(tag))
        if st == SS_ENOMEM:
            return False
        _check(st)
        return True

    def step(self, iters: int = 4) -> int:
        n = C.c_int32()
        _check(_lib.ss_engine_step(self._h, int(iters), C.byref(n)))
        return n.value

    def poll(self, cap: int = 4096):
        tags = np.zeros(cap, dtype=np.int64)
        probs = np.zeros(cap, dtype=np.int32)
        info = (SolveInfo * cap)()
        n = C.c_int32()
        _check(_lib.ss_engine_poll(self._h, cap, _ptr(tags, C.c_int64), _ptr(probs, C.c_int32), info,
                                   C.byref(n)))
        return [(int(tags[i]), int(probs[i]), info[i].as_dict()) for i in range(n.value)]

    def usage(self):
        n = C.c_int32()
        b = C.c_int64()
        _check(_lib.ss_engine_usage(self._h, C.byref(n), C.byref(b)))
        return n.value, b.value

    def close(self):
        if self._h:
            _lib.ss_engine_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def proxy_error(stamp_next: Stamp, op_next: Operator, u, problems, stream=None) -> np.ndarray:
    """Exact proxy error |f - L u^N|_2 / |f|_2 of every problem (Sec. 10.1, Lemma ProxyError).

    ``stamp_next`` and ``op_next`` are built on the same problems at level N + 1; ``u`` is the
    device complex128 tensor of the level-N solutions in the level-N stamp's canonical order."""
    vals = problems.f_hat if isinstance(problems, Batch) else \
        _c128(np.concatenate([np.asarray(p.f_hat) for p in problems]))
    if vals is None or len(vals) != 2 * stamp_next.n_f:
        raise SparseSpecError(SS_EINVAL, "one f_hat coefficient per forcing frequency of the build is needed")
    err = np.zeros(stamp_next.n_prob, dtype=np.float64)
    _check(_lib.ss_proxy_error(stamp_next._h, op_next._h, C.c_void_p(u.data_ptr()), int(u.numel()),
                               _ptr(vals, C.c_double), _ptr(err, C.c_double), C.c_void_p(_stream(stream))))
    return err


def solve(d, a_freqs, a_hat, f_freqs, f_hat, level, tol=1e-12, precision="fp64", max_iter=2000, flags=0,
          want_keys=True, x0=None):
    """One-shot solve from host data; returns ``(u_hat, keys, info)`` in canonical order.
    ``x0``: optional initial guess (complex, |S^N| entries in canonical order)."""
    af = _i16(np.asarray(a_freqs).reshape(-1, d))
    ff = _i16(np.asarray(f_freqs).reshape(-1, d))
    ah = _c128(a_hat)
    fh = _c128(f_hat)
    n = C.c_int64()
    info = SolveInfo()
    _check(_lib.ss_solve(d, len(af), _ptr(af, C.c_int16), _ptr(ah, C.c_double), len(ff), _ptr(ff, C.c_int16),
                         _ptr(fh, C.c_double), int(level), float(tol), PRECISION[precision], int(max_iter),
                         int(flags), None, 0, C.byref(n), None, None, C.byref(info)))
    u = np.zeros(n.value, dtype=np.complex128)
    x0v = None
    if x0 is not None:
        x0v = _c128(x0)
        if len(x0v) != 2 * n.value:
            raise SparseSpecError(SS_EINVAL, "x0 needs |S^N| entries")
    keys = np.zeros((n.value, d), dtype=np.int16) if want_keys else None
    _check(_lib.ss_solve(d, len(af), _ptr(af, C.c_int16), _ptr(ah, C.c_double), len(ff), _ptr(ff, C.c_int16),
                         _ptr(fh, C.c_double), int(level), float(tol), PRECISION[precision], int(max_iter),
                         int(flags), _ptr(x0v, C.c_double) if x0v is not None else None, n.value, C.byref(n),
                         _ptr(u.view(np.float64), C.c_double),
                         _ptr(keys, C.c_int16) if want_keys else None, C.byref(info)))
    return u, keys, info.as_dict()


def version() -> str:
    return _lib.ss_version().decode()


def memory_stats() -> dict:
    """The library's device allocator: bytes held, bytes cached, driver allocations so far."""
    live, cached, allocs = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    _check(_lib.ss_memory_stats(C.byref(live), C.byref(cached), C.byref(allocs)))
    return {"live_bytes": live.value, "cached_bytes": cached.value, "driver_allocs": allocs.value}


class BatchSolution:
    """Device-resident solutions of ``solve_batch`` (every problem's u in canonical order)."""

    def __init__(self, handle, n_prob: int):
        self._h = handle
        n = C.c_int64()
        self.offsets = np.zeros(n_prob + 1, dtype=np.int64)
        _check(_lib.ss_batch_size(self._h, C.byref(n), _ptr(self.offsets, C.c_int64)))
        self.n_total = n.value

    def solution(self, out=None, stream=None):
        """u of all problems concatenated (complex128 tensor on the current device)."""
        import torch
        if out is None:
            out = torch.empty(self.n_total, dtype=torch.complex128, device="cuda")
        _check(_lib.ss_batch_solution(self._h, C.c_void_p(out.data_ptr()), C.c_void_p(_stream(stream))))
        return out

    def close(self):
        if self._h:
            _lib.ss_free_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(problems, tol: float, precision="fp64", max_iter: int = 1000, flags: int = 0, parts: int = 4):
    """Whole path for a batch of one dimension from host data, split into ``parts`` concurrent
    parts.  Returns (BatchSolution, [info dict per problem]); raises on errors other than
    non-convergence (then the infos tell which problems missed the tolerance)."""
    b = _batch(problems)
    if b.a_hat is None or b.f_hat is None:
        raise SparseSpecError(SS_EINVAL, "a_hat and f_hat of every problem are needed")
    info = (SolveInfo * b.n_prob)()
    h = C.c_void_p()
    st = _lib.ss_solve_batch(b.n_prob, b.d, _ptr(b.n_a, C.c_int32), _ptr(b.a_freqs, C.c_int16),
                             _ptr(b.a_hat, C.c_double), _ptr(b.n_f, C.c_int32), _ptr(b.f_freqs, C.c_int16),
                             _ptr(b.f_hat, C.c_double), _ptr(b.level, C.c_int32), float(tol),
                             PRECISION[precision], int(max_iter), int(flags), int(parts), C.byref(h), info)
    if st not in (SS_OK, SS_ENOCONV, SS_EBREAKDOWN) or not h.value:
        _check(st)
    return BatchSolution(h, b.n_prob), [i.as_dict() for i in info]


def lattice_modulus(expansion: int, n: int, sigma: float) -> int:
    """The smallest prime greater than max(expansion, n^2 / sigma) (Lemma RandomRank1Lattice)."""
    M = C.c_int64(0)
    _check(_lib.ss_lattice_modulus(int(expansion), int(n), float(sigma), C.byref(M)))
    return M.value
