"""ctypes front of the plain-C oracle (c/dcs_oracle.c).  TEST INFRASTRUCTURE ONLY."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "c", "dcs_oracle.c")
LIB = os.path.join(_HERE, "c", "libdcs_oracle.so")

_u64p = C.POINTER(C.c_uint64)
_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)
_f32p = C.POINTER(C.c_float)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        l = C.CDLL(LIB)
        l.orc_sector_create.restype = C.c_void_p
        l.orc_sector_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _i32p]
        l.orc_sector_free.argtypes = [C.c_void_p]
        l.orc_dim.restype = C.c_uint64
        l.orc_dim.argtypes = [C.c_void_p]
        l.orc_rank.restype = C.c_uint64
        l.orc_rank.argtypes = [C.c_void_p, C.c_uint64]
        l.orc_unrank.restype = C.c_uint64
        l.orc_unrank.argtypes = [C.c_void_p, C.c_uint64]
        l.orc_rank_batch.argtypes = [C.c_void_p, _u64p, _u64p, C.c_int64]
        l.orc_unrank_batch.argtypes = [C.c_void_p, _u64p, _u64p, C.c_int64]
        l.orc_iter_create.restype = C.c_void_p
        l.orc_iter_create.argtypes = [C.c_void_p]
        l.orc_iter_free.argtypes = [C.c_void_p]
        l.orc_iter_next.restype = C.c_int64
        l.orc_iter_next.argtypes = [C.c_void_p, C.c_void_p, _u64p, C.c_int64]
        hx = [C.c_void_p, C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p]
        l.orc_hx_range.argtypes = hx + [_f64p, C.c_int, C.c_uint64, C.c_int64, _f64p]
        l.orc_hx_rows.argtypes = hx + [_f64p, C.c_int, _u64p, C.c_int64, _f64p]
        l.orc_hx_rows_xf32.argtypes = hx + [_f32p, C.c_int, _u64p, C.c_int64, _f64p]
        l.orc_bond_sums.argtypes = [C.c_void_p, C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_int,
                                    C.c_uint64, C.c_int64, _f64p, _f64p, _f64p]
        l.orc_num_threads.restype = C.c_int
        l.orc_set_threads.argtypes = [C.c_int]
        _lib = l
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


class NativeSector:
    """Sector index of the C oracle (closed form, eq. index; nested generation)."""

    def __init__(self, Q: int, L: int, n: int, split):
        self.Q, self.L, self.n = Q, L, n
        self.split = list(split)
        sp = np.asarray(self.split, dtype=np.int32)
        self._h = lib().orc_sector_create(Q, L, n, len(sp), _p(sp, _i32p))
        if not self._h:
            raise ValueError("oracle rejected the sector parameters")
        self.dim = int(lib().orc_dim(self._h))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_sector_free(self._h)
            self._h = None

    def rank(self, states) -> np.ndarray:
        st = np.ascontiguousarray(states, dtype=np.uint64)
        out = np.empty_like(st)
        lib().orc_rank_batch(self._h, _p(st, _u64p), _p(out, _u64p), len(st))
        return out

    def unrank(self, idx) -> np.ndarray:
        ix = np.ascontiguousarray(idx, dtype=np.uint64)
        out = np.empty_like(ix)
        lib().orc_unrank_batch(self._h, _p(ix, _u64p), _p(out, _u64p), len(ix))
        return out

    def iterate(self, chunk: int = 1 << 22):
        """Canonical order by nested generation, yielded in chunks of packed states."""
        it = lib().orc_iter_create(self._h)
        try:
            buf = np.empty(chunk, dtype=np.uint64)
            while True:
                got = lib().orc_iter_next(self._h, it, _p(buf, _u64p), chunk)
                if got == 0:
                    return
                yield buf[:got].copy()
        finally:
            lib().orc_iter_free(it)


class NativeTerms:
    def __init__(self, bonds, jxy, jz, h=None):
        self.bi = np.ascontiguousarray([b[0] for b in bonds], dtype=np.int32)
        self.bj = np.ascontiguousarray([b[1] for b in bonds], dtype=np.int32)
        self.jxy = np.ascontiguousarray(jxy, dtype=np.float64)
        self.jz = np.ascontiguousarray(jz, dtype=np.float64)
        self.h = None if h is None else np.ascontiguousarray(h, dtype=np.float64)

    def args(self):
        hp = _p(self.h, _f64p) if self.h is not None else None
        return [len(self.bi), _p(self.bi, _i32p), _p(self.bj, _i32p), _p(self.jxy, _f64p),
                _p(self.jz, _f64p), hp]


def hx_range(sec: NativeSector, terms: NativeTerms, x: np.ndarray, first: int = 0,
             count: int | None = None) -> np.ndarray:
    """Rows [first, first+count) of H x (FP64).  x is [dim] or [dim, k] FP64."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    k = 1 if x.ndim == 1 else x.shape[1]
    count = sec.dim - first if count is None else count
    y = np.empty((count, k))
    lib().orc_hx_range(sec._h, *terms.args(), _p(x, _f64p), k, first, count, _p(y, _f64p))
    return y[:, 0] if x.ndim == 1 else y


def hx_rows(sec: NativeSector, terms: NativeTerms, x: np.ndarray, rows) -> np.ndarray:
    """(H x) at the listed rows, FP64.  x may be FP64 or FP32 ([dim] or [dim, k])."""
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    k = 1 if x.ndim == 1 else x.shape[1]
    y = np.empty((len(rows), k))
    if x.dtype == np.float32:
        xf = np.ascontiguousarray(x)
        lib().orc_hx_rows_xf32(sec._h, *terms.args(), _p(xf, _f32p), k, _p(rows, _u64p),
                               len(rows), _p(y, _f64p))
    else:
        xd = np.ascontiguousarray(x, dtype=np.float64)
        lib().orc_hx_rows(sec._h, *terms.args(), _p(xd, _f64p), k, _p(rows, _u64p),
                          len(rows), _p(y, _f64p))
    return y[:, 0] if x.ndim == 1 else y


def bond_sums(sec: NativeSector, bonds, x: np.ndarray, g: np.ndarray, fields: bool = False,
              first: int = 0, count: int | None = None):
    """(g . A_b x, g . Z_b x) for every listed bond (and g . Sz_i x for every site if
    ``fields``), summed over rows [first, first+count) and all columns; FP64.
    x and g are [dim] or [dim, k] FP64."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    if x.shape != g.shape:
        raise ValueError("x and g differ in shape")
    k = 1 if x.ndim == 1 else x.shape[1]
    count = sec.dim - first if count is None else count
    bi = np.ascontiguousarray([b[0] for b in bonds], dtype=np.int32)
    bj = np.ascontiguousarray([b[1] for b in bonds], dtype=np.int32)
    gxy = np.zeros(max(len(bonds), 1))
    gz = np.zeros(max(len(bonds), 1))
    gh = np.zeros(sec.L) if fields else None
    lib().orc_bond_sums(sec._h, len(bonds), _p(bi, _i32p), _p(bj, _i32p), _p(x, _f64p), _p(g, _f64p),
                        k, first, count, _p(gxy, _f64p), _p(gz, _f64p),
                        _p(gh, _f64p) if fields else None)
    return gxy[:len(bonds)], gz[:len(bonds)], gh


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls (on the calling thread)."""
    lib().orc_set_threads(int(n))
