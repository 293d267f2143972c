"""ctypes binding of the plain FP64 C oracle of the auxiliary-grid AMG method.

TEST INFRASTRUCTURE ONLY: imported by the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py``. The HIP library never imports, links or executes anything here.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, INVALID, NOMEM, NOT_SPD, BREAKDOWN, NOCONV = 0, 1, 2, 4, 5, 6


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        p, i64, i32, d = C.c_void_p, C.c_int64, C.c_int, C.c_double
        L.orc_depth.argtypes = [i64, i32, C.POINTER(i32), C.POINTER(i32)]
        L.orc_depth_dim.argtypes = [i64, i32, i32, C.POINTER(i32), C.POINTER(i32)]
        L.orc_cell_index.argtypes = [i64, p, p, i32, p]
        L.orc_cell_index.restype = None
        L.orc_cell_index_dim.argtypes = [i64, i32, p, p, i32, p]
        L.orc_cell_index_dim.restype = None
        L.orc_setup.argtypes = [i64, p, p, p, p, p, i32, i32, i32, C.POINTER(p)]
        L.orc_setup_dim.argtypes = [i64, i32, p, p, p, p, p, i32, i32, i32, C.POINTER(p)]
        L.orc_dim.argtypes = [p]
        L.orc_free.argtypes = [p]
        L.orc_free.restype = None
        L.orc_solve.argtypes = [p, p, p, d, i32, i32, C.POINTER(i32), C.POINTER(d)]
        L.orc_apply_precond.argtypes = [p, p, p]
        L.orc_num_levels.argtypes = [p]
        L.orc_level_info.argtypes = [p, i32, C.POINTER(i64), C.POINTER(i32), C.POINTER(i64), C.POINTER(i32)]
        L.orc_export_level.argtypes = [p, i32, p, p, p, p, p, p, p]
        L.orc_smooth.argtypes = [p, i32, p, p, i32]
        L.orc_set_block_smoother.argtypes = [p, i32]
        L.orc_level_spmv.argtypes = [p, i32, p, p]
        L.orc_restrict.argtypes = [p, i32, p, p]
        L.orc_prolong_add.argtypes = [p, i32, p, p]
        L.orc_test_force_restart.argtypes = [i32]
        L.orc_test_force_restart.restype = None
        L.orc_nlpcg_test.argtypes = [i64, p, p, p, p, i32, i32, p]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def depth(n: int, coarse_max: int = 64, dim: int = 2):
    L, kc = C.c_int(), C.c_int()
    nlev = lib().orc_depth_dim(n, dim, coarse_max, C.byref(L), C.byref(kc))
    return nlev, L.value, kc.value


def cell_index(coords: np.ndarray, box, L: int) -> np.ndarray:
    """Level-L cell of each point; coords (n, 2) or (n, 3), box {a1, b1, a2, b2[, a3, b3]}."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    bx = np.ascontiguousarray(box, dtype=np.float64)
    out = np.empty(len(coords), dtype=np.int32)
    lib().orc_cell_index_dim(len(coords), coords.shape[1], _ptr(coords), _ptr(bx), L, _ptr(out))
    return out


class Oracle:
    """Setup + solve of the oracle. Vectors are float64 numpy arrays in the caller's numbering (fine level) or the
    lexicographic cell numbering (quadtree levels)."""

    def __init__(self, coords, row_ptr, col, val, box=None, coarse_max=64, inner_iters=2, sweeps=1):
        self._keep = [np.ascontiguousarray(coords, dtype=np.float64), np.ascontiguousarray(row_ptr, dtype=np.int64),
                      np.ascontiguousarray(col, dtype=np.int32), np.ascontiguousarray(val, dtype=np.float64)]
        bx = None if box is None else np.ascontiguousarray(box, dtype=np.float64)
        self.n = len(self._keep[0])
        self.dim = self._keep[0].shape[1] if self._keep[0].ndim == 2 else 2
        self.slots = 27 if self.dim == 3 else 9
        h = C.c_void_p()
        st = lib().orc_setup_dim(self.n, self.dim, *[_ptr(a) for a in self._keep], _ptr(bx), coarse_max,
                                 inner_iters, sweeps, C.byref(h))
        if st != OK:
            raise OracleError(st, "orc_setup")
        self._h = h
        self.num_levels = lib().orc_num_levels(h)

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    __del__ = close

    def level_info(self, level: int):
        n, k, ovf, L = C.c_int64(), C.c_int(), C.c_int64(), C.c_int()
        st = lib().orc_level_info(self._h, level, C.byref(n), C.byref(k), C.byref(ovf), C.byref(L))
        if st != OK:
            raise OracleError(st, "orc_level_info")
        return dict(n=n.value, k=k.value, ovf_nnz=ovf.value, L=L.value)

    def export_level(self, level: int) -> dict:
        info = self.level_info(level)
        n = info["n"]
        out = dict(info)
        out["agg"] = np.empty(n, dtype=np.int32)
        out["color"] = np.empty(n, dtype=np.uint8)
        if level == 0:
            st = lib().orc_export_level(self._h, 0, _ptr(out["agg"]), _ptr(out["color"]), None, None, None, None,
                                        None)
        else:
            out["aj"] = np.empty((n, self.slots), dtype=np.int32)
            out["ax"] = np.empty((n, self.slots), dtype=np.float64)
            out["ovf_ptr"] = np.empty(n + 1, dtype=np.int64)
            out["ovf_col"] = np.empty(info["ovf_nnz"], dtype=np.int32)
            out["ovf_val"] = np.empty(info["ovf_nnz"], dtype=np.float64)
            st = lib().orc_export_level(self._h, level, *[_ptr(out[k]) for k in
                                                           ("agg", "color", "aj", "ax", "ovf_ptr", "ovf_col",
                                                            "ovf_val")])
        if st != OK:
            raise OracleError(st, "orc_export_level")
        return out

    def solve(self, b, tol=1e-8, max_iters=1000, mmax=1):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty(self.n)
        it, rr = C.c_int(), C.c_double()
        st = lib().orc_solve(self._h, _ptr(b), _ptr(x), tol, max_iters, mmax, C.byref(it), C.byref(rr))
        return x, dict(status=st, iters=it.value, relres=rr.value)

    def apply_precond(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty(self.n)
        st = lib().orc_apply_precond(self._h, _ptr(r), _ptr(z))
        if st != OK:
            raise OracleError(st, "orc_apply_precond")
        return z

    def set_block_smoother(self, on=True):
        """Exact solves of the cells' diagonal blocks in the fine smoother (cells of at most 32 unknowns)."""
        st = lib().orc_set_block_smoother(self._h, 1 if on else 0)
        if st:
            raise OracleError(st, "orc_set_block_smoother")

    def smooth(self, level, f, x, forward=True):
        f = np.ascontiguousarray(f, dtype=np.float64)
        x = np.array(x, dtype=np.float64, copy=True)
        st = lib().orc_smooth(self._h, level, _ptr(f), _ptr(x), 1 if forward else 0)
        if st != OK:
            raise OracleError(st, "orc_smooth")
        return x

    def restrict(self, level, r):
        """P^t r from level `level` to level + 1."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        fc = np.empty(self.level_info(level + 1)["n"])
        st = lib().orc_restrict(self._h, level, _ptr(r), _ptr(fc))
        if st != OK:
            raise OracleError(st, "orc_restrict")
        return fc

    def prolong_add(self, level, e, u):
        """u + P e from level + 1 to level `level` (u is not modified)."""
        e = np.ascontiguousarray(e, dtype=np.float64)
        u = np.array(u, dtype=np.float64, copy=True)
        st = lib().orc_prolong_add(self._h, level, _ptr(e), _ptr(u))
        if st != OK:
            raise OracleError(st, "orc_prolong_add")
        return u

    def solve_forced_restart(self, b, at_iter, tol=1e-8, max_iters=1000, mmax=1):
        """solve() with the recurrence residual zeroed once after `at_iter` iterations (test of the restart)."""
        lib().orc_test_force_restart(int(at_iter))
        try:
            return self.solve(b, tol=tol, max_iters=max_iters, mmax=mmax)
        finally:
            lib().orc_test_force_restart(0)

    def spmv(self, level, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty_like(x)
        st = lib().orc_level_spmv(self._h, level, _ptr(x), _ptr(y))
        if st != OK:
            raise OracleError(st, "orc_level_spmv")
        return y


def setup_problem(prob, **kw) -> Oracle:
    return Oracle(prob.coords, prob.row_ptr, prob.col, prob.val, box=prob.box, **kw)


def nlpcg_test(row_ptr, col, val, f, nsteps, mode):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    va = np.ascontiguousarray(val, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    u = np.empty(len(f))
    st = lib().orc_nlpcg_test(len(f), _ptr(rp), _ptr(ci), _ptr(va), _ptr(f), nsteps, mode, _ptr(u))
    if st != OK:
        raise OracleError(st, "orc_nlpcg_test")
    return u
