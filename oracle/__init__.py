"""CPU FP64 oracle for the staggered operator and its CG solve.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The library under
`paper_1311_2719_amd/` never imports it, and the two share no code: the
operator and the solver here are written from the paper
(P. Majumdar, arXiv:1311.2719, Sec. 3 for the matrix-vector routine, Sec. 4
for the conjugate-gradient loop) and from the textbook definitions, in plain
C (`stag_oracle.c`, loaded through ctypes) and NumPy (`dense.py`,
`free_field.py`).

Array conventions: links complex128 [V,4,3,3], vectors complex128 [V,3],
sites lexicographic s = x + Lx*(y + Ly*(z + Lz*t)).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stag_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

EVEN, ODD, ALL = 0, 1, 2


class CGResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("rr", ctypes.c_double),
        ("bb", ctypes.c_double),
        ("true_rel", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


def build(force: bool = False) -> str:
    """Compile stag_oracle.c with gcc into liboracle.so (OpenMP on)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            I32, I64, D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
            lib.orc_dslash.argtypes = [P, I32, P, P, P, I32]
            lib.orc_dslash.restype = ctypes.c_int
            lib.orc_dslash_sites.argtypes = [P, I32, P, P, P, I64, P]
            lib.orc_dslash_sites.restype = ctypes.c_int
            lib.orc_apply_normal.argtypes = [P, I32, P, D, I32, P, P]
            lib.orc_apply_normal.restype = ctypes.c_int
            lib.orc_true_residual.argtypes = [P, I32, P, D, I32, P, P]
            lib.orc_true_residual.restype = D
            lib.orc_cg_solve.argtypes = [P, I32, P, D, D, I32, I32, I32, P, P, P, P]
            lib.orc_cg_solve.restype = ctypes.c_int
            lib.orc_cg_pass.argtypes = [P, I32, P, D, D, I32, I32, P, P, P]
            lib.orc_cg_pass.restype = ctypes.c_int
            lib.orc_cg_full.argtypes = [P, I32, P, D, D, I32, I32, P, P, P]
            lib.orc_cg_full.restype = ctypes.c_int
            lib.orc_max_threads.argtypes = []
            lib.orc_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    if d.shape != (4,):
        raise ValueError("dims must be 4 integers")
    return d


def _c128(a, shape):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.shape != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), a.shape))
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().orc_max_threads())


def dslash(dims, U, chi, out_parity=ALL, antiperiodic_t=True, out=None):
    """(D chi)(x) on the sites of out_parity; other sites of `out` untouched
    (zero when `out` is not given)."""
    lib = _load()
    L = _dims(dims)
    V = int(np.prod(L))
    U = _c128(U, (V, 4, 3, 3))
    chi = _c128(chi, (V, 3))
    res = np.zeros((V, 3), np.complex128) if out is None else out
    if res.dtype != np.complex128 or not res.flags.c_contiguous or res.shape != (V, 3):
        raise ValueError("out must be contiguous complex128 [V,3]")
    rc = lib.orc_dslash(_ptr(L), int(bool(antiperiodic_t)), _ptr(U), _ptr(chi), _ptr(res), int(out_parity))
    if rc != 0:
        raise ValueError("orc_dslash rejected its arguments")
    return res


def dslash_sites(dims, U, chi, sites, antiperiodic_t=True):
    """(D chi) at the listed lexicographic sites: complex128 [n,3]."""
    lib = _load()
    L = _dims(dims)
    V = int(np.prod(L))
    U = _c128(U, (V, 4, 3, 3))
    chi = _c128(chi, (V, 3))
    s = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    out = np.zeros((s.size, 3), np.complex128)
    rc = lib.orc_dslash_sites(_ptr(L), int(bool(antiperiodic_t)), _ptr(U), _ptr(chi), _ptr(s), s.size, _ptr(out))
    if rc != 0:
        raise ValueError("orc_dslash_sites rejected its arguments")
    return out


def apply_normal(dims, U, m, v, parity=ALL, antiperiodic_t=True):
    """(m^2 - D^2) v on the sites of `parity` (zero elsewhere)."""
    lib = _load()
    L = _dims(dims)
    V = int(np.prod(L))
    U = _c128(U, (V, 4, 3, 3))
    v = _c128(v, (V, 3))
    out = np.zeros((V, 3), np.complex128)
    rc = lib.orc_apply_normal(_ptr(L), int(bool(antiperiodic_t)), _ptr(U), float(m), int(parity), _ptr(v), _ptr(out))
    if rc != 0:
        raise ValueError("orc_apply_normal rejected its arguments")
    return out


def true_residual(dims, U, m, b, x, parity=ALL, antiperiodic_t=True) -> float:
    """||b - (m^2 - D^2) x|| / ||b|| over the sites of `parity`, FP64."""
    lib = _load()
    L = _dims(dims)
    V = int(np.prod(L))
    U = _c128(U, (V, 4, 3, 3))
    b = _c128(b, (V, 3))
    x = _c128(x, (V, 3))
    return float(lib.orc_true_residual(_ptr(L), int(bool(antiperiodic_t)), _ptr(U), float(m), int(parity), _ptr(b), _ptr(x)))


def cg_solve(dims, U, m, b, tol=1e-10, maxiter=20000, max_restarts=10,
             parity=ALL, want_y=False, antiperiodic_t=True):
    """Even-odd CG of the paper's Sec. 4 loop on each parity system, with
    FP64 true-residual restarts.  Returns (x, y or None, info dict)."""
    lib = _load()
    L = _dims(dims)
    V = int(np.prod(L))
    U = _c128(U, (V, 4, 3, 3))
    b = _c128(b, (V, 3))
    x = np.zeros((V, 3), np.complex128)
    y = np.zeros((V, 3), np.complex128) if want_y else None
    res = CGResult()
    rc = lib.orc_cg_solve(_ptr(L), int(bool(antiperiodic_t)), _ptr(U), float(m), float(tol),
                          int(maxiter), int(max_restarts), int(parity), _ptr(b), _ptr(x),
                          _ptr(y) if y is not None else None, ctypes.byref(res))
    if rc < 0:
        raise ValueError("orc_cg_solve rejected its arguments")
    return x, y, res.as_dict()


def cg_pass(dims, U, m, b, tol, maxiter, parity, antiperiodic_t=True):
    """One CG pass from x = 0 on one parity system with no restart; with
    tol = 0 it returns the maxiter-th iterate."""
    lib = _load()
    L = _dims(dims)
    V = int(np.prod(L))
    U = _c128(U, (V, 4, 3, 3))
    b = _c128(b, (V, 3))
    x = np.zeros((V, 3), np.complex128)
    res = CGResult()
    rc = lib.orc_cg_pass(_ptr(L), int(bool(antiperiodic_t)), _ptr(U), float(m), float(tol),
                         int(maxiter), int(parity), _ptr(b), _ptr(x), ctypes.byref(res))
    if rc < 0:
        raise ValueError("orc_cg_pass rejected its arguments")
    return x, res.as_dict()


def cg_full(dims, U, m, b, tol=1e-13, maxiter=100000, max_restarts=20,
            x0=None, antiperiodic_t=True):
    """Textbook CG on the whole lattice with true-residual restarts, used for
    the tight reference solution."""
    lib = _load()
    L = _dims(dims)
    V = int(np.prod(L))
    U = _c128(U, (V, 4, 3, 3))
    b = _c128(b, (V, 3))
    x = np.zeros((V, 3), np.complex128) if x0 is None else np.array(_c128(x0, (V, 3)))
    res = CGResult()
    rc = lib.orc_cg_full(_ptr(L), int(bool(antiperiodic_t)), _ptr(U), float(m), float(tol),
                         int(maxiter), int(max_restarts), _ptr(b), _ptr(x), ctypes.byref(res))
    if rc < 0:
        raise ValueError("orc_cg_full rejected its arguments")
    return x, res.as_dict()
