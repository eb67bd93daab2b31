"""Thin ctypes binding of libspand (names follow include/spand.h).

Argument marshalling only: every step of the factorization, the apply and PCG
runs inside the HIP library.  Device arrays are torch tensors on a ROCm device
(``float64``, column-major n x nrhs for vectors, i.e. shape (nrhs, n) contiguous
or a Fortran-ordered (n, nrhs) view); host arrays are numpy arrays.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import re
import sys
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

SPAND_FP64, SPAND_FP32, SPAND_BF16X3 = 0, 1, 2
SPAND_ORTHS, SPAND_IN, SPAND_INS = 0, 1, 2
VARIANTS = {"OrthS": SPAND_ORTHS, "In": SPAND_IN, "InS": SPAND_INS}
STATUS = {0: "SPAND_OK", 1: "SPAND_E_INVALID", 2: "SPAND_E_NOT_SPD", 3: "SPAND_E_NOCONV",
          4: "SPAND_E_NOMEM", 5: "SPAND_E_HIP", 6: "SPAND_E_STATE", 7: "SPAND_E_BREAKDOWN"}


class SpandError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Tuning(C.Structure):
    _fields_ = [("chol_group", C.c_int32), ("fuse128_min", C.c_int32), ("gemm_syrk", C.c_int32),
                ("cpqr_big_min", C.c_int32), ("gemm_chol", C.c_int32), ("gemm_scale", C.c_int32),
                ("reserved", C.c_int32 * 2)]
    KEYS = ("chol_group", "fuse128_min", "gemm_syrk", "cpqr_big_min", "gemm_chol", "gemm_scale")

    def as_dict(self):
        return {k: getattr(self, k) for k in self.KEYS}


class Stats(C.Structure):
    _fields_ = [("t_analyze", C.c_double), ("t_factor", C.c_double), ("t_solve", C.c_double),
                ("n", C.c_int64), ("levels", C.c_int32), ("n_steps", C.c_int32), ("last_iters", C.c_int32),
                ("s_top", C.c_int32), ("m_F", C.c_int64), ("schur_flops", C.c_double),
                ("schur_seconds", C.c_double), ("fail_step", C.c_int32), ("fail_cluster", C.c_int32),
                ("fail_phase", C.c_int32), ("cpqr_one_launch_steps", C.c_int32),
                ("step_phase_seconds", (C.c_double * 4) * 32), ("step_m_F", C.c_int64 * 32),
                ("cpqr_flops", C.c_double), ("cpqr_seconds", C.c_double), ("cpqr_launches", C.c_int64),
                ("apply_bytes", C.c_double), ("apply_seconds", C.c_double), ("apply_calls", C.c_int64),
                ("apply_graph", C.c_int32), ("cpqr_lds_slot_interfaces", C.c_int32), ("cpqr_interfaces", C.c_int64 * 4),
                ("apply_interfaces", C.c_int64 * 3), ("pcg_replacements", C.c_int64),
                ("cpqr_big_interfaces", C.c_int64), ("apply_scratch_per_rhs", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_
             if k not in ("step_phase_seconds", "step_m_F", "cpqr_interfaces",
                          "apply_interfaces")}
        d["cpqr_interfaces"] = [int(v) for v in self.cpqr_interfaces]
        d["apply_interfaces"] = [int(v) for v in self.apply_interfaces]
        L = max(0, min(32, int(self.n_steps)))
        d["step_phase_seconds"] = [[self.step_phase_seconds[t][q] for q in range(4)] for t in range(L)]
        d["step_m_F"] = [int(self.step_m_F[t]) for t in range(L)]
        return d


def library_path() -> str:
    return os.path.join(HERE, "libspand.so")


def load_library():
    """Load libspand.so; raises if it has not been built (no fallback exists)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1901_02971_amd.build`")
    lib = C.CDLL(path)
    P = C.c_void_p
    i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
    sig = {
        "spand_analyze": (i32, [i64, P, P, i32, P, i32, C.POINTER(P)]),
        "spand_factor": (i32, [P, P, f64, i32, i32]),
        "spand_solve": (i32, [P, i32, P, P, f64, i32, P, P]),
        "spand_apply": (i32, [P, i32, P, P]),
        "spand_set_stream": (i32, [P, P]),
        "spand_set_apply_graph": (i32, [P, i32]),
        "spand_get_stats": (i32, [P, C.POINTER(Stats)]),
        "spand_set_tuning": (i32, [P, C.POINTER(Tuning)]),
        "spand_get_tuning": (i32, [P, C.POINTER(Tuning)]),
        "spand_set_variant": (i32, [P, i32]),
        "spand_get_variant": (i32, [P, C.POINTER(i32)]),
        "spand_autotune": (i32, [P, P, f64, i32, i32, i32, i32, C.POINTER(Tuning)]),
        "spand_get_ordering": (i32, [P, P, P, P]),
        "spand_get_permutation": (i32, [P, P]),
        "spand_step_counts": (i32, [P, i32, P]),
        "spand_step_structure": (i32, [P, i32, P, P, P, P, P]),
        "spand_step_ranks": (i32, [P, i32, P, P]),
        "spand_factor_batch": (i32, [i32, P, P, f64, i32, i32]),
        "spand_solve_batch": (i32, [i32, P, i32, P, P, f64, i32, P, P]),
        "spand_error_string": (C.c_char_p, [P]),
        "spand_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def exported_symbols():
    """Function names declared in include/spand.h."""
    hdr = os.path.join(os.path.dirname(HERE), "include", "spand.h")
    src = open(hdr).read()
    return sorted(set(re.findall(r"\b(spand_[a-z_]+)\s*\(", src)))


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()  # torch tensor


def _dev_vec(t, n):
    """Validate a float64 device tensor holding an n x nrhs column-major block."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("expected a float64 tensor on the GPU")
    if t.dim() == 1:
        if t.numel() != n:
            raise ValueError("length mismatch")
        return 1
    if t.dim() == 2 and t.shape[1] == n and t.is_contiguous():
        return t.shape[0]          # (nrhs, n) row-major = n x nrhs column-major
    if t.dim() == 2 and t.shape[0] == n and t.t().is_contiguous():
        return t.shape[1]          # Fortran-ordered (n, nrhs)
    raise ValueError("expected shape (nrhs, n) contiguous or a column-major (n, nrhs) view")


# Every live handle, so that they are all released while the HIP runtime and torch
# are still up: the exit hook below is registered when this module is imported,
# after torch, so it runs before torch's own exit hooks.
_LIVE = weakref.WeakSet()


def close_all():
    """Release every open handle (idempotent)."""
    for s in list(_LIVE):
        s.close()


atexit.register(close_all)


class Solver:
    """One spaND handle: analyze on construction, then factor / solve / apply.

    Call close() (or use the Solver as a context manager) to release the handle's
    device memory deterministically; handles still open at interpreter exit are
    released by an exit hook, never from a finalizer during shutdown."""

    def __init__(self, n, rowptr, colind, coords, levels):
        lib = load_library()
        self._lib = lib
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        colind = np.ascontiguousarray(colind, dtype=np.int32)
        if coords is None:   # graph separator: no geometry
            dim = 0
        else:
            coords = np.ascontiguousarray(coords, dtype=np.float64)
            dim = coords.shape[1] if coords.ndim == 2 else 1
        self.n = int(n)
        self.levels = int(levels)
        h = C.c_void_p()
        st = lib.spand_analyze(self.n, _ptr(rowptr), _ptr(colind), dim, _ptr(coords), self.levels, C.byref(h))
        if st != 0:
            raise SpandError(st, lib.spand_error_string(None).decode())
        self._h = h
        _LIVE.add(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @classmethod
    def from_problem(cls, problem, levels, geometry=True):
        """geometry=False analyzes the graph alone (level-structure separator)."""
        return cls(problem.n, problem.rowptr, problem.colind, problem.coords if geometry else None, levels)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.spand_destroy(self._h)
            self._h = None
        _LIVE.discard(self)

    def __del__(self):
        # during interpreter shutdown the exit hook has already released the handle;
        # device teardown from a finalizer at that point is not safe
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise SpandError(st, self._lib.spand_error_string(self._h).decode())

    def set_stream(self, stream):
        """Run on a torch.cuda.Stream (or raw hipStream_t int); None = default stream."""
        raw = None if stream is None else (stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        self._check(self._lib.spand_set_stream(self._h, raw))

    def set_apply_graph(self, enable):
        """Replay the PCG apply as a captured HIP graph (default) or launch it eagerly."""
        self._check(self._lib.spand_set_apply_graph(self._h, 1 if enable else 0))

    def factor(self, values, tol, skip=0, prec=SPAND_FP64):
        import torch
        if not (isinstance(values, torch.Tensor) and values.is_cuda and values.dtype == torch.float64
                and values.is_contiguous()):
            raise TypeError("values must be a contiguous float64 GPU tensor")
        self._check(self._lib.spand_factor(self._h, _ptr(values), float(tol), int(skip), int(prec)))

    def solve(self, b, x, rtol=1e-12, maxit=500, check=True):
        nrhs = _dev_vec(b, self.n)
        if _dev_vec(x, self.n) != nrhs:
            raise ValueError("b and x differ in nrhs")
        iters = np.zeros(nrhs, dtype=np.int32)
        relres = np.zeros(nrhs, dtype=np.float64)
        st = self._lib.spand_solve(self._h, nrhs, _ptr(b), _ptr(x), float(rtol), int(maxit), _ptr(iters), _ptr(relres))
        if check and st != 0:
            self._check(st)
        return iters, relres, st

    def apply(self, r, z):
        nrhs = _dev_vec(r, self.n)
        self._check(self._lib.spand_apply(self._h, nrhs, _ptr(r), _ptr(z)))

    def tuning(self):
        t = Tuning()
        self._check(self._lib.spand_get_tuning(self._h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = Tuning()
        self._check(self._lib.spand_get_tuning(self._h, C.byref(t)))
        for k, v in kw.items():
            if k not in Tuning.KEYS:
                raise KeyError(k)
            setattr(t, k, int(v))
        self._check(self._lib.spand_set_tuning(self._h, C.byref(t)))

    def set_variant(self, variant):
        """spand_set_variant: "OrthS" (default), "In" or "InS" for the later factors."""
        self._check(self._lib.spand_set_variant(self._h, VARIANTS[variant] if isinstance(variant, str) else int(variant)))

    def variant(self):
        v = C.c_int32()
        self._check(self._lib.spand_get_variant(self._h, C.byref(v)))
        return {num: name for name, num in VARIANTS.items()}[v.value]

    def autotune(self, values, tol, skip=0, prec=SPAND_FP64, nrhs=1, reps=2):
        """spand_autotune: choose the kernel shapes on this matrix; the handle ends
        factored with them.  Returns the chosen tuning."""
        import torch
        if not (isinstance(values, torch.Tensor) and values.is_cuda and values.dtype == torch.float64
                and values.is_contiguous()):
            raise TypeError("values must be a contiguous float64 GPU tensor")
        t = Tuning()
        self._check(self._lib.spand_autotune(self._h, _ptr(values), float(tol), int(skip), int(prec), int(nrhs),
                                             int(reps), C.byref(t)))
        return t.as_dict()

    def stats(self):
        s = Stats()
        self._check(self._lib.spand_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def ordering(self):
        S = np.zeros(self.n, np.int64)
        L = np.zeros(self.n, np.int64)
        R = np.zeros(self.n, np.int64)
        self._check(self._lib.spand_get_ordering(self._h, _ptr(S), _ptr(L), _ptr(R)))
        return S, L, R

    def permutation(self):
        perm = np.zeros(self.n, np.int64)
        self._check(self._lib.spand_get_permutation(self._h, _ptr(perm)))
        return perm

    def step_counts(self, step):
        c = np.zeros(6, np.int64)
        self._check(self._lib.spand_step_counts(self._h, int(step), _ptr(c)))
        return dict(nc=int(c[0]), ne=int(c[1]), nb=int(c[2]), na=int(c[3]), level=int(c[4]), nenb=int(c[5]))

    def step_structure(self, step):
        c = self.step_counts(step)
        keys = np.zeros((c["nc"], 3), np.int64)
        parent = np.zeros(c["nc"], np.int32)
        colour = np.zeros(c["nc"], np.int32)
        before = np.zeros((c["nb"], 2), np.int32)
        after = np.zeros((c["na"], 2), np.int32)
        self._check(self._lib.spand_step_structure(self._h, int(step), _ptr(keys), _ptr(parent), _ptr(colour),
                                                   _ptr(before), _ptr(after)))
        return dict(keys=keys, parent=parent, colour=colour, before=before, after=after, **c)

    def step_ranks(self, step):
        c = self.step_counts(step)
        sizes = np.zeros(c["nc"], np.int32)
        ranks = np.zeros(c["nc"], np.int32)
        self._check(self._lib.spand_step_ranks(self._h, int(step), _ptr(sizes), _ptr(ranks)))
        return sizes, ranks


def factor_batch(solvers, values, tol, skip=0, prec=SPAND_FP64):
    """spand_factor_batch over the handles of `solvers` (distinct Solver objects) with
    values[q] a contiguous float64 GPU tensor for solvers[q]."""
    import torch
    if len(solvers) != len(values) or not solvers:
        raise ValueError("one values tensor per solver")
    for v in values:
        if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float64 and v.is_contiguous()):
            raise TypeError("values must be contiguous float64 GPU tensors")
    lib = load_library()
    P = len(solvers)
    hs = (C.c_void_p * P)(*[s._h.value for s in solvers])
    vp = (C.c_void_p * P)(*[v.data_ptr() for v in values])
    st = lib.spand_factor_batch(P, hs, vp, float(tol), int(skip), int(prec))
    if st != 0:
        raise SpandError(st, lib.spand_error_string(None).decode())


def solve_batch(solvers, b, x, rtol=1e-12, maxit=500, check=True):
    """spand_solve_batch: b[q], x[q] device blocks of solvers[q] (same nrhs for all).
    Returns (iters, relres, status) with iters, relres of shape (P, nrhs)."""
    if not (len(solvers) == len(b) == len(x)) or not solvers:
        raise ValueError("one b and one x per solver")
    nrhs = _dev_vec(b[0], solvers[0].n)
    for s, bq, xq in zip(solvers, b, x):
        if _dev_vec(bq, s.n) != nrhs or _dev_vec(xq, s.n) != nrhs:
            raise ValueError("every problem must have the same nrhs")
    lib = load_library()
    P = len(solvers)
    hs = (C.c_void_p * P)(*[s._h.value for s in solvers])
    bp = (C.c_void_p * P)(*[t.data_ptr() for t in b])
    xp = (C.c_void_p * P)(*[t.data_ptr() for t in x])
    iters = np.zeros((P, nrhs), dtype=np.int32)
    relres = np.zeros((P, nrhs), dtype=np.float64)
    st = lib.spand_solve_batch(P, hs, nrhs, bp, xp, float(rtol), int(maxit), _ptr(iters), _ptr(relres))
    if check and st != 0:
        raise SpandError(st, lib.spand_error_string(None).decode())
    return iters, relres, st
