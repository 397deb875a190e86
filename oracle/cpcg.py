"""The timed CPU baseline: sparse FP64 Jacobi-preconditioned CG in plain C with OpenMP
(``cpcg.c``; test infrastructure only, shares no code with the GPU library).

``solve_batch`` runs stamp, index and solve for every problem of a batch on ``threads`` OpenMP
threads and returns the per-problem phase times, sizes, iterations and residuals, plus the
solutions in canonical slot order when asked.  ``build`` compiles ``libcpcg.so`` with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpcg.c")
LIB = os.path.join(HERE, "libcpcg.so")


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("iters", C.c_int32), ("status", C.c_int32),
                ("rel_residual", C.c_double), ("stamp_ms", C.c_double), ("index_ms", C.c_double),
                ("solve_ms", C.c_double), ("matvec_ms", C.c_double)]


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", SRC, "-o", tmp,
           "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed on cpcg.c:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = C.CDLL(LIB)
        P = C.c_void_p
        lib.cpcg_solve_batch.argtypes = [C.c_int, C.c_int, P, P, P, P, P, P, P, C.c_double, C.c_int, C.c_int, C.c_int,
                                         P, P, C.c_int64, C.POINTER(Info), C.POINTER(C.c_int)]
        lib.cpcg_solve_batch.restype = C.c_int
        _lib = lib
    return _lib


def _p(a):
    return C.c_void_p(a.ctypes.data)


def solve_batch(problems, tol: float, threads: int, max_iter: int = 10000, matvec_reps: int = 0,
                want_u: bool = False):
    """Returns (status, infos: list of dicts, threads used, u list or None).  ``problems`` carry
    ``d, a_freqs, a_hat`` (full support closed under negation, with 0), ``f_freqs, f_hat, level``."""
    lib = _load()
    d = int(problems[0].d)
    n_a = np.array([len(p.a_freqs) for p in problems], dtype=np.int32)
    n_f = np.array([len(p.f_freqs) for p in problems], dtype=np.int32)
    lev = np.array([int(p.level) for p in problems], dtype=np.int32)
    af = np.ascontiguousarray(np.concatenate([np.asarray(p.a_freqs).reshape(-1, d) for p in problems]), np.int16)
    ff = np.ascontiguousarray(np.concatenate([np.asarray(p.f_freqs).reshape(-1, d) for p in problems]), np.int16)
    ah = np.ascontiguousarray(np.concatenate([np.asarray(p.a_hat) for p in problems]), np.complex128)
    fh = np.ascontiguousarray(np.concatenate([np.asarray(p.f_hat) for p in problems]), np.complex128)
    infos = (Info * len(problems))()
    used = C.c_int(0)
    u = u_off = None
    cap = 0
    if want_u:
        cap = 0
        for p in problems:   # bound on |S^N|: every key is f plus at most N elements of supp(a)
            cap += len(p.f_freqs) * (len(p.a_freqs) ** int(p.level))
        cap = min(cap, 1 << 26)
        u = np.zeros(cap, dtype=np.complex128)
        u_off = np.zeros(len(problems) + 1, dtype=np.int64)
    st = lib.cpcg_solve_batch(len(problems), d, _p(n_a), _p(af), _p(ah), _p(n_f), _p(ff), _p(fh), _p(lev),
                              float(tol), int(max_iter), int(threads), int(matvec_reps),
                              _p(u) if want_u else None, _p(u_off) if want_u else None, cap, infos, C.byref(used))
    out = [{f: getattr(i, f) for f, _ in Info._fields_} for i in infos]
    sols = [u[u_off[i]:u_off[i + 1]].copy() for i in range(len(problems))] if want_u else None
    return st, out, used.value, sols
