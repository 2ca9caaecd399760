"""ctypes binding of libstagcg (C ABI in include/stagcg.h).

Argument marshalling only: every step of D_slash and of the CG solves runs
in the library's HIP kernels.  PyTorch supplies the device memory (one arena
tensor per context, plus the caller's field tensors) and the HIP stream.

Fermion fields on the device are torch.complex128 tensors in the library's
even-odd layout, shape (2, 3, V/2): [parity][colour][checkerboard site].
`Context.pack` / `Context.unpack` convert from / to the lexicographic
(V, 3) layout that the oracle and the input generators use.
"""

from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstagcg.so")

OK, PENDING = 0, 1
ERRORS = {
    -1: "EINVAL", -2: "ENOMEM", -3: "ENOENT", -4: "EBUSY", -5: "EAGAIN",
    -6: "ENOCONV", -7: "EBREAKDOWN", -8: "ENONFINITE", -9: "EHIP", -10: "ECANCELED",
}
EINVAL, ENOMEM, ENOENT, EBUSY, EAGAIN, ENOCONV, EBREAKDOWN, ENONFINITE, EHIP, ECANCELED = range(-1, -11, -1)
EVEN, ODD, ALL = 0, 1, 2
FP64, FP32_RU, FP16_RU = 0, 1, 2
F64, F32, F16 = 0, 1, 2  # storage precision of a fermion field (stag_dslash, stag_convert_fermion)
SPINOR_BYTES = {F64: 48, F32: 24, F16: 16}  # per site
FP16_DELTA_MIN = 0.01

_lock = threading.Lock()
_lib = None


class StagError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "ERR"), code, msg))
        self.code = code


class CGParams(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("maxiter", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("parity", ctypes.c_int32),
        ("max_restarts", ctypes.c_int32),
        ("delta", ctypes.c_double),
    ]


class MDParams(ctypes.Structure):
    _fields_ = [
        ("beta", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("nsteps", ctypes.c_int32),
        ("maxiter", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("t_antiperiodic", ctypes.c_int32),
    ]


class MDInfo(ctypes.Structure):
    _fields_ = [
        ("kinetic", ctypes.c_double * 2),
        ("gauge_action", ctypes.c_double * 2),
        ("fermion_action", ctypes.c_double * 2),
        ("delta_h", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("cg_iters", ctypes.c_int32),
        ("solves", ctypes.c_int32),
    ]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if isinstance(v, ctypes.Array) else v
        return d


class CGInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("reliable_updates", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("true_rel_resid", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("queue_seconds", ctypes.c_double),
        ("iters_parity", ctypes.c_int32 * 2),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["iters_parity"] = [int(v) for v in self.iters_parity]
        return d


def load():
    """Open libstagcg.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libstagcg.so is not built (%s); run `python -m paper_1311_2719_amd.build`" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        P, I32, I64, SZ, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_uint64
        sig = {
            "stag_create": ([ctypes.c_int, P, SZ, P, ctypes.POINTER(P)], ctypes.c_int),
            "stag_destroy": ([P], ctypes.c_int),
            "stag_last_error": ([P], ctypes.c_char_p),
            "stag_arena_usage": ([P, ctypes.POINTER(SZ), ctypes.POINTER(SZ)], ctypes.c_int),
            "stag_set_gauge": ([P, P, P, I32, I32, ctypes.POINTER(I32)], ctypes.c_int),
            "stag_free_gauge": ([P, I32], ctypes.c_int),
            "stag_gauge_dims": ([P, I32, P], ctypes.c_int),
            "stag_gauge_link_rows": ([P, I32, ctypes.POINTER(I32)], ctypes.c_int),
            "stag_pack_fermion": ([P, P, P, P, P], ctypes.c_int),
            "stag_unpack_fermion": ([P, P, P, P, P], ctypes.c_int),
            "stag_dslash": ([P, I32, I32, I64, I64, P, P, I32, I32, I32, P], ctypes.c_int),
            "stag_convert_fermion": ([P, P, P, I32, P, I32, P], ctypes.c_int),
            "stag_cg_solve": ([P, I32, ctypes.POINTER(CGParams), P, P, P, I32, P, ctypes.POINTER(CGInfo)],
                              ctypes.c_int),
            "stag_cg_solve_batch": ([P, I32, I32, ctypes.POINTER(CGParams), P, P, P, ctypes.POINTER(CGInfo)],
                                    ctypes.c_int),
            "stag_cg_solve_noalloc": ([P, I32, ctypes.POINTER(CGParams), P, P, P, P, ctypes.POINTER(CGInfo)],
                                      ctypes.c_int),
            "stag_fermion_force": ([P, I32, P, P, ctypes.c_double, I32, P], ctypes.c_int),
            "stag_gauge_force": ([P, P, P, ctypes.c_double, P, ctypes.c_double, I32, P], ctypes.c_int),
            "stag_pseudofermion": ([P, I32, P, P, ctypes.c_double, P], ctypes.c_int),
            "stag_md_trajectory": ([P, P, P, P, P, ctypes.POINTER(MDParams), P, ctypes.POINTER(MDInfo)],
                                   ctypes.c_int),
            "stag_submit": ([P, I32, ctypes.POINTER(CGParams), P, P, ctypes.POINTER(U64)], ctypes.c_int),
            "stag_poll": ([P, U64, ctypes.POINTER(CGInfo)], ctypes.c_int),
            "stag_wait": ([P, U64, ctypes.POINTER(CGInfo)], ctypes.c_int),
            "stag_release_ticket": ([P, U64], ctypes.c_int),
            "stag_serve_config": ([P, I32, I32, I32], ctypes.c_int),
            "stag_tune_info": ([P, I32, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32),
                                ctypes.POINTER(I32)], ctypes.c_int),
            "stag_cg_tune_info": ([P, I32, I32, I32] + [ctypes.POINTER(I32)] * 6, ctypes.c_int),
            "stag_version": ([], ctypes.c_char_p),
            "stag_set_gauge_wilson": ([P, P, P, I32, I32, ctypes.POINTER(I32)], ctypes.c_int),
            "stag_pack_spinor": ([P, P, P, P, P], ctypes.c_int),
            "stag_unpack_spinor": ([P, P, P, P, P], ctypes.c_int),
            "stag_wilson_dslash": ([P, I32, I32, P, P, P], ctypes.c_int),
            "stag_wilson_solve": ([P, I32, ctypes.c_double, ctypes.c_double, I32, P, P, P, ctypes.POINTER(CGInfo)],
                                  ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
        return lib


def exported_symbols():
    """Names of the C ABI entry points the binding expects."""
    return [
        "stag_create", "stag_destroy", "stag_last_error", "stag_arena_usage", "stag_set_gauge",
        "stag_free_gauge", "stag_gauge_dims", "stag_gauge_link_rows", "stag_pack_fermion", "stag_unpack_fermion", "stag_dslash",
        "stag_convert_fermion", "stag_cg_solve", "stag_cg_solve_noalloc", "stag_cg_solve_batch", "stag_submit", "stag_poll", "stag_wait",
        "stag_release_ticket", "stag_serve_config", "stag_fermion_force", "stag_gauge_force",
        "stag_pseudofermion", "stag_md_trajectory", "stag_tune_info", "stag_cg_tune_info", "stag_version",
        "stag_set_gauge_wilson", "stag_pack_spinor", "stag_unpack_spinor", "stag_wilson_dslash",
        "stag_wilson_solve",
    ]


def _check(rc: int, what: str) -> int:
    if rc < 0:
        msg = load().stag_last_error(None)
        raise StagError(rc, "%s: %s" % (what, msg.decode() if msg else ""))
    return rc


def _torch():
    import torch

    return torch


def params(mass, tol=1e-10, maxiter=20000, precision=FP64, parity=ALL, max_restarts=10, delta=0.0) -> CGParams:
    """CG parameters; delta <= 0 leaves the reliable-update threshold to the library default."""
    return CGParams(float(mass), float(tol), int(maxiter), int(precision), int(parity), int(max_restarts),
                    float(delta))


@dataclass
class Field:
    gauge_id: int
    dims: tuple

    @property
    def volume(self):
        return int(np.prod(self.dims))


class Context:
    """A library context on one GPU.  `arena_bytes` of device memory are
    allocated once with torch and handed to the library, which sub-allocates
    every gauge field and workspace from it."""

    def __init__(self, device: int = 0, arena_bytes: int = 4 << 30, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the stagcg library runs on the GPU only")
        self.lib = load()
        self.device = int(device)
        self.torch_device = torch.device("cuda", self.device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.torch_device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.torch_device)
        h = ctypes.c_void_p()
        _check(self.lib.stag_create(self.device, self.arena.data_ptr(), int(arena_bytes),
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "stag_create")
        self.h = h
        self.fields = {}
        # tensors a queued request borrows (b, x), held until its ticket is
        # released so that Python cannot free them while the server uses them
        self._borrowed = {}

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            _check(self.lib.stag_destroy(self.h), "stag_destroy")
            self.h = None
            self._borrowed = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def arena_usage(self):
        used, total = ctypes.c_size_t(), ctypes.c_size_t()
        _check(self.lib.stag_arena_usage(self.h, ctypes.byref(used), ctypes.byref(total)), "stag_arena_usage")
        return used.value, total.value

    # -- gauge fields --------------------------------------------------------
    def set_gauge(self, dims, links, antiperiodic_t=True) -> Field:
        """links: complex128 [V,4,3,3], numpy (host) or a torch CUDA tensor."""
        return self._register(self.lib.stag_set_gauge, "stag_set_gauge", dims, links, antiperiodic_t)

    def set_gauge_wilson(self, dims, links, antiperiodic_t=True) -> Field:
        """The same links registered for the Wilson-fermion operator."""
        return self._register(self.lib.stag_set_gauge_wilson, "stag_set_gauge_wilson", dims, links, antiperiodic_t)

    def _register(self, fn, name, dims, links, antiperiodic_t):
        torch = _torch()
        d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
        gid = ctypes.c_int32()
        if isinstance(links, torch.Tensor):
            if links.dtype != torch.complex128 or not links.is_contiguous():
                raise ValueError("links must be contiguous complex128")
            ptr, on_dev = links.data_ptr(), int(links.is_cuda)
            keep = links
        else:
            keep = np.ascontiguousarray(links, dtype=np.complex128)
            ptr, on_dev = keep.ctypes.data, 0
        V = int(np.prod(d))
        if tuple(keep.shape) != (V, 4, 3, 3):
            raise ValueError("links must have shape (V,4,3,3)")
        _check(fn(self.h, d.ctypes.data, ctypes.c_void_p(ptr), on_dev, int(bool(antiperiodic_t)), ctypes.byref(gid)),
               name)
        f = Field(gid.value, tuple(int(v) for v in d))
        self.fields[gid.value] = f
        return f

    def link_rows(self, field: Field) -> int:
        """Link rows the library stores for `field` (2: third row rebuilt, or 3)."""
        rows = ctypes.c_int32()
        _check(self.lib.stag_gauge_link_rows(self.h, field.gauge_id, ctypes.byref(rows)), "stag_gauge_link_rows")
        return rows.value

    def free_gauge(self, field: Field):
        _check(self.lib.stag_free_gauge(self.h, field.gauge_id), "stag_free_gauge")
        self.fields.pop(field.gauge_id, None)

    # -- fields ----------------------------------------------------------------
    def new_fermion(self, field: Field, precision=F64):
        """A zero field on the device in the even-odd layout: complex128 or
        complex64 (2, 3, V/2) for F64 / F32, 16-byte records uint8 (2, V/2, 16)
        for F16."""
        torch = _torch()
        vh = field.volume // 2
        if precision == F16:
            return torch.zeros((2, vh, 16), dtype=torch.uint8, device=self.torch_device)
        dt = torch.complex128 if precision == F64 else torch.complex64
        return torch.zeros((2, 3, vh), dtype=dt, device=self.torch_device)

    def convert(self, field: Field, inp, out, in_precision, out_precision, stream=None):
        """out = inp converted between storage precisions (device tensors)."""
        for t, pr in ((inp, in_precision), (out, out_precision)):
            self._check_prec(field, t, pr, device=True)
        d = np.asarray(field.dims, dtype=np.int32)
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(self.lib.stag_convert_fermion(self.h, d.ctypes.data, ctypes.c_void_p(inp.data_ptr()), int(in_precision),
                                             ctypes.c_void_p(out.data_ptr()), int(out_precision), s),
               "stag_convert_fermion")
        return out

    def _check_prec(self, field, t, precision, device):
        """t: a contiguous torch CUDA tensor (device) or numpy array (host)
        holding one full-lattice field of `precision`."""
        torch = _torch()
        need = field.volume // 2 * 2 * SPINOR_BYTES[int(precision)]
        if device:
            ok = isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous() and t.numel() * t.element_size() == need
        else:
            ok = isinstance(t, np.ndarray) and t.flags.c_contiguous and t.nbytes == need
        if not ok:
            raise ValueError("expected a contiguous %s field of %d bytes" % ("device" if device else "host", need))

    def pack(self, field: Field, lex):
        """(V,3) complex128 (numpy or torch) -> device even-odd tensor (2,3,V/2)."""
        torch = _torch()
        if not isinstance(lex, torch.Tensor):
            lex = torch.from_numpy(np.ascontiguousarray(lex, dtype=np.complex128))
        lex = lex.to(self.torch_device).contiguous()
        if lex.shape != (field.volume, 3) or lex.dtype != torch.complex128:
            raise ValueError("expected complex128 (V,3)")
        eo = self.new_fermion(field)
        d = np.asarray(field.dims, dtype=np.int32)
        _check(self.lib.stag_pack_fermion(self.h, d.ctypes.data, ctypes.c_void_p(lex.data_ptr()),
                                          ctypes.c_void_p(eo.data_ptr()), None), "stag_pack_fermion")
        return eo

    def unpack(self, field: Field, eo):
        """device even-odd (2,3,V/2) -> device lexicographic (V,3)."""
        torch = _torch()
        self._check_eo(field, eo)
        lex = torch.empty((field.volume, 3), dtype=torch.complex128, device=self.torch_device)
        d = np.asarray(field.dims, dtype=np.int32)
        _check(self.lib.stag_unpack_fermion(self.h, d.ctypes.data, ctypes.c_void_p(eo.data_ptr()),
                                            ctypes.c_void_p(lex.data_ptr()), None), "stag_unpack_fermion")
        return lex

    def _check_eo(self, field, t):
        torch = _torch()
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
                and tuple(t.shape) == (2, 3, field.volume // 2)):
            raise ValueError("expected a contiguous complex128 CUDA tensor of shape (2,3,V/2)")

    # -- Wilson spin-colour vectors ---------------------------------------------------
    def new_spinor(self, field: Field):
        torch = _torch()
        return torch.zeros((2, 12, field.volume // 2), dtype=torch.complex128, device=self.torch_device)

    def _check_spinor(self, field, t):
        torch = _torch()
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
                and tuple(t.shape) == (2, 12, field.volume // 2)):
            raise ValueError("expected a contiguous complex128 CUDA tensor of shape (2,12,V/2)")

    def pack_spinor(self, field: Field, lex):
        """(V,4,3) complex128 (numpy or torch) -> device even-odd tensor (2,12,V/2)."""
        torch = _torch()
        if not isinstance(lex, torch.Tensor):
            lex = torch.from_numpy(np.ascontiguousarray(lex, dtype=np.complex128))
        lex = lex.to(self.torch_device).contiguous()
        if tuple(lex.shape) != (field.volume, 4, 3) or lex.dtype != torch.complex128:
            raise ValueError("expected complex128 (V,4,3)")
        eo = self.new_spinor(field)
        d = np.asarray(field.dims, dtype=np.int32)
        _check(self.lib.stag_pack_spinor(self.h, d.ctypes.data, ctypes.c_void_p(lex.data_ptr()),
                                         ctypes.c_void_p(eo.data_ptr()), None), "stag_pack_spinor")
        return eo

    def unpack_spinor(self, field: Field, eo):
        """device even-odd (2,12,V/2) -> device lexicographic (V,4,3)."""
        torch = _torch()
        self._check_spinor(field, eo)
        lex = torch.empty((field.volume, 4, 3), dtype=torch.complex128, device=self.torch_device)
        d = np.asarray(field.dims, dtype=np.int32)
        _check(self.lib.stag_unpack_spinor(self.h, d.ctypes.data, ctypes.c_void_p(eo.data_ptr()),
                                           ctypes.c_void_p(lex.data_ptr()), None), "stag_unpack_spinor")
        return lex

    def wilson_dslash(self, field: Field, inp, out, out_parity=ALL):
        """out = H inp on the sites of out_parity (Wilson hopping term)."""
        self._check_spinor(field, inp)
        self._check_spinor(field, out)
        _check(self.lib.stag_wilson_dslash(self.h, field.gauge_id, int(out_parity), ctypes.c_void_p(inp.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), None), "stag_wilson_dslash")
        return out

    def wilson_solve(self, field: Field, b, x, kappa, tol=1e-10, maxiter=20000, check=True):
        """M x = b, M = 1 - kappa H, by CG on the even-odd normal equations."""
        self._check_spinor(field, b)
        self._check_spinor(field, x)
        info = CGInfo()
        rc = self.lib.stag_wilson_solve(self.h, field.gauge_id, float(kappa), float(tol), int(maxiter),
                                        ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), None,
                                        ctypes.byref(info))
        if check:
            _check(rc, "stag_wilson_solve")
        d = info.as_dict()
        d["rc"] = rc
        return d

    # -- operator and solves ------------------------------------------------------
    def dslash(self, field: Field, inp, out, out_parity=ALL, offset=0, count=-1, accumulate=False, stream=None,
               precision=F64):
        """out (+)= D inp on a site range of out_parity.  inp/out: torch CUDA
        tensors (asynchronous on the library's stream), or numpy arrays on
        the host (copied in and out; returns when out is complete)."""
        on_device = not isinstance(inp, np.ndarray)
        self._check_prec(field, inp, precision, on_device)
        self._check_prec(field, out, precision, on_device)
        if isinstance(out, np.ndarray) != isinstance(inp, np.ndarray):
            raise ValueError("inp and out must both be host arrays or both device tensors")
        ptr = (lambda a: a.ctypes.data) if not on_device else (lambda t: t.data_ptr())
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(self.lib.stag_dslash(self.h, field.gauge_id, int(out_parity), int(offset), int(count),
                                    ctypes.c_void_p(ptr(inp)), ctypes.c_void_p(ptr(out)),
                                    int(bool(accumulate)), int(precision), int(on_device), s), "stag_dslash")
        return out

    def cg_solve(self, field: Field, b, x, y=None, check=True, **kw):
        """Solve on device tensors (b, x, y complex128 (2,3,V/2) on the GPU) or
        on host arrays (numpy complex128 (2,3,V/2): copied in and out)."""
        p = params(**kw)
        on_device = not isinstance(b, np.ndarray)
        for t in (b, x) + ((y,) if y is not None else ()):
            if on_device:
                self._check_eo(field, t)
            else:
                self._check_prec(field, t, F64, device=False)
        ptr = (lambda a: a.ctypes.data) if not on_device else (lambda t: t.data_ptr())
        info = CGInfo()
        rc = self.lib.stag_cg_solve(self.h, field.gauge_id, ctypes.byref(p), ctypes.c_void_p(ptr(b)),
                                    ctypes.c_void_p(ptr(x)),
                                    ctypes.c_void_p(ptr(y)) if y is not None else None, int(on_device), None,
                                    ctypes.byref(info))
        if check:
            _check(rc, "stag_cg_solve")
        d = info.as_dict()
        d["rc"] = rc
        return d

    def cg_solve_noalloc(self, field: Field, b, x, y=None, check=True, **kw):
        """The solve on device tensors with the library's fixed workspace
        (stag_cg_solve_noalloc): no memory is allocated by the call."""
        p = params(**kw)
        for t in (b, x) + ((y,) if y is not None else ()):
            self._check_eo(field, t)
        info = CGInfo()
        rc = self.lib.stag_cg_solve_noalloc(self.h, field.gauge_id, ctypes.byref(p), ctypes.c_void_p(b.data_ptr()),
                                            ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(y.data_ptr()) if y is not None else None, None,
                                            ctypes.byref(info))
        if check:
            _check(rc, "stag_cg_solve_noalloc")
        d = info.as_dict()
        d["rc"] = rc
        return d

    def cg_solve_batch(self, field: Field, bs, xs, plist, check=True):
        n = len(bs)
        if not (len(xs) == n == len(plist)):
            raise ValueError("bs, xs and params must have the same length")
        for t in list(bs) + list(xs):
            self._check_eo(field, t)
        P = (CGParams * n)(*plist)
        B = (ctypes.c_void_p * n)(*[t.data_ptr() for t in bs])
        X = (ctypes.c_void_p * n)(*[t.data_ptr() for t in xs])
        infos = (CGInfo * n)()
        rc = self.lib.stag_cg_solve_batch(self.h, field.gauge_id, n, P, ctypes.cast(B, ctypes.c_void_p),
                                          ctypes.cast(X, ctypes.c_void_p), None, infos)
        if check:
            _check(rc, "stag_cg_solve_batch")
        out = [i.as_dict() for i in infos]
        for d in out:
            d["rc"] = rc
        return out

    # -- molecular dynamics ----------------------------------------------------
    def fermion_force(self, field: Field, w, force=None, coeff=1.0, accumulate=False, stream=None):
        """force (+)= coeff * F, the pseudofermion force from w (device even-odd
        field: the solution on the even sites, D_oe of it on the odd sites).
        force: complex128 (V, 4, 3, 3) on the device (allocated if None)."""
        torch = _torch()
        self._check_eo(field, w)
        if force is None:
            force = torch.zeros((field.volume, 4, 3, 3), dtype=torch.complex128, device=self.torch_device)
        if not (isinstance(force, torch.Tensor) and force.is_cuda and force.dtype == torch.complex128
                and force.is_contiguous() and tuple(force.shape) == (field.volume, 4, 3, 3)):
            raise ValueError("force must be a contiguous complex128 CUDA tensor (V, 4, 3, 3)")
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(self.lib.stag_fermion_force(self.h, field.gauge_id, ctypes.c_void_p(w.data_ptr()),
                                           ctypes.c_void_p(force.data_ptr()), float(coeff), int(bool(accumulate)),
                                           s), "stag_fermion_force")
        return force

    def _check_links(self, dims, t, what):
        torch = _torch()
        V = int(np.prod(dims))
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
                and tuple(t.shape) == (V, 4, 3, 3)):
            raise ValueError("%s must be a contiguous complex128 CUDA tensor (V, 4, 3, 3)" % what)

    def gauge_force(self, dims, links, beta, force=None, coeff=1.0, accumulate=False, stream=None):
        """force (+)= coeff * F_G for device links (V, 4, 3, 3)."""
        torch = _torch()
        d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
        self._check_links(d, links, "links")
        if force is None:
            force = torch.zeros_like(links)
        self._check_links(d, force, "force")
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(self.lib.stag_gauge_force(self.h, d.ctypes.data, ctypes.c_void_p(links.data_ptr()), float(beta),
                                         ctypes.c_void_p(force.data_ptr()), float(coeff), int(bool(accumulate)), s),
               "stag_gauge_force")
        return force

    def pseudofermion(self, field: Field, chi, mass, phi=None):
        """phi = m chi - D chi on the even sites (device even-odd fields)."""
        self._check_eo(field, chi)
        if phi is None:
            phi = self.new_fermion(field)
        self._check_eo(field, phi)
        _check(self.lib.stag_pseudofermion(self.h, field.gauge_id, ctypes.c_void_p(chi.data_ptr()),
                                           ctypes.c_void_p(phi.data_ptr()), float(mass), None), "stag_pseudofermion")
        return phi

    def md_trajectory(self, dims, links, momenta, phi, beta, mass, eps, nsteps, tol=1e-10, maxiter=20000,
                      precision=FP64, antiperiodic_t=True, check=True):
        """One leapfrog trajectory; links and momenta (V, 4, 3, 3) device tensors
        are updated in place; phi a device even-odd pseudofermion."""
        d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
        self._check_links(d, links, "links")
        self._check_links(d, momenta, "momenta")
        p = MDParams(float(beta), float(mass), float(eps), float(tol), int(nsteps), int(maxiter), int(precision),
                     int(bool(antiperiodic_t)))
        info = MDInfo()
        rc = self.lib.stag_md_trajectory(self.h, d.ctypes.data, ctypes.c_void_p(links.data_ptr()),
                                         ctypes.c_void_p(momenta.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                                         ctypes.byref(p), None, ctypes.byref(info))
        if check:
            _check(rc, "stag_md_trajectory")
        out = info.as_dict()
        out["rc"] = rc
        return out

    # -- serving ---------------------------------------------------------------
    def serve_config(self, slots_per_field=16, epoch_iters=16, queue_capacity=4096):
        _check(self.lib.stag_serve_config(self.h, int(slots_per_field), int(epoch_iters), int(queue_capacity)),
               "stag_serve_config")

    def submit(self, field: Field, b, x, **kw) -> int:
        p = params(**kw)
        self._check_eo(field, b)
        self._check_eo(field, x)
        t = ctypes.c_uint64()
        _check(self.lib.stag_submit(self.h, field.gauge_id, ctypes.byref(p), ctypes.c_void_p(b.data_ptr()),
                                    ctypes.c_void_p(x.data_ptr()), ctypes.byref(t)), "stag_submit")
        self._borrowed[t.value] = (b, x)
        return t.value

    def poll(self, ticket: int):
        info = CGInfo()
        rc = self.lib.stag_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(info))
        if rc == PENDING:
            return None
        if rc in (ENOENT, EINVAL):
            _check(rc, "stag_poll")
        d = info.as_dict()
        d["rc"] = rc
        return d

    def wait(self, ticket: int):
        info = CGInfo()
        rc = self.lib.stag_wait(self.h, ctypes.c_uint64(ticket), ctypes.byref(info))
        if rc in (ENOENT, EINVAL):
            _check(rc, "stag_wait")
        d = info.as_dict()
        d["rc"] = rc
        return d

    def release(self, ticket: int):
        _check(self.lib.stag_release_ticket(self.h, ctypes.c_uint64(ticket)), "stag_release_ticket")
        self._borrowed.pop(int(ticket), None)

    def tune_info(self, field: Field, precision=FP64, nrhs=1):
        v = [ctypes.c_int32() for _ in range(4)]
        _check(self.lib.stag_tune_info(self.h, field.gauge_id, int(precision), int(nrhs),
                                       *[ctypes.byref(t) for t in v]), "stag_tune_info")
        return {"lanes_per_site": v[0].value, "block": v[1].value, "rhs_tile": v[2].value,
                "use_tables": v[3].value}

    def cg_tune_info(self, field: Field, precision=FP64, nrhs=1):
        """The CG step shape tuned for (field, precision, nrhs) once such a
        solve has run (StagError ENOENT before)."""
        v = [ctypes.c_int32() for _ in range(6)]
        _check(self.lib.stag_cg_tune_info(self.h, field.gauge_id, int(precision), int(nrhs),
                                          *[ctypes.byref(t) for t in v]), "stag_cg_tune_info")
        return {"lanes_per_site": v[0].value, "block": v[1].value, "rhs_tile": v[2].value,
                "use_tables": v[3].value, "reduction_kernel": v[4].value, "shared_links": v[5].value}


def version() -> str:
    return load().stag_version().decode()
