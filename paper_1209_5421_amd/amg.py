"""Python binding of the quadamg C ABI (include/quadamg.h): argument marshalling only.

Every step of setup and solve runs in the HIP kernels of libquadamg.so; torch is used for device memory and the
stream handle. If the library is missing or no GPU is present, calls raise instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libquadamg.so")

OK, INVALID, NOMEM, DEVICE, NOT_SPD, BREAKDOWN, NOCONV = range(7)
STATUS = {0: "AMG_OK", 1: "AMG_ERR_INVALID", 2: "AMG_ERR_NOMEM", 3: "AMG_ERR_DEVICE", 4: "AMG_ERR_NOT_SPD",
          5: "AMG_ERR_BREAKDOWN", 6: "AMG_ERR_NOCONV"}
EXPORTED = ["amg_default_options", "amg_setup", "amg_setup3d", "amg_update_values", "amg_solve", "amg_free", "amg_set_precision", "amg_set_stream",
            "amg_solve_batch", "amg_solve_batch_noalloc", "amg_cache_control", "amg_estimate_bytes", "amg_hierarchy_bytes", "amg_num_levels", "amg_level_info",
            "amg_export_level", "amg_export_level_f32", "amg_apply_precond", "amg_level_smooth", "amg_level_spmv",
            "amg_kernel_timing_enable", "amg_kernel_timing_read", "amg_engine_info", "amg_p1_mesh_create",
            "amg_p1_mesh_pattern", "amg_p1_assemble", "amg_p1_mesh_free", "amg_status_string"]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("coarse_max", C.c_int32), ("inner_iters", C.c_int32),
                ("sweeps", C.c_int32), ("outer_mmax", C.c_int32), ("max_iters", C.c_int32),
                ("engine", C.c_int32), ("batch", C.c_int32), ("smoother", C.c_int32), ("box", C.POINTER(C.c_double)),
                ("stream", C.c_void_p), ("alloc", C.c_void_p), ("dealloc", C.c_void_p), ("ctx", C.c_void_p)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEALLOC_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class TorchAllocator:
    """amg_options.alloc / dealloc backed by torch's caching allocator: the hierarchy's device memory then comes from
    (and returns to) the same cache as the caller's tensors, on the hierarchy's device and stream. The callback
    objects must outlive every hierarchy set up with them (Hierarchy keeps a reference)."""

    def __init__(self, device, stream=None):
        import torch
        self.device = torch.device(device).index or 0
        self.stream = stream
        self.live = 0  # blocks handed out and not yet returned

        def _alloc(nbytes, _ctx):
            try:
                s = self.stream if self.stream is not None else torch.cuda.current_stream(self.device)
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, s)
                self.live += 1
                return p
            except Exception:
                return None

        def _dealloc(ptr, _ctx):
            torch.cuda.caching_allocator_delete(ptr)
            self.live -= 1

        self._alloc = ALLOC_FN(_alloc)
        self._dealloc = DEALLOC_FN(_dealloc)

    def install(self, o):
        o.alloc = C.cast(self._alloc, C.c_void_p)
        o.dealloc = C.cast(self._dealloc, C.c_void_p)
        o.ctx = None


class Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32), ("relres", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AMGError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libquadamg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
    L = C.CDLL(path)
    p, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.amg_default_options.argtypes = [C.POINTER(Options)]
    L.amg_default_options.restype = None
    L.amg_setup.argtypes = [i64, p, p, p, p, i64, C.POINTER(Options), C.POINTER(p)]
    L.amg_setup3d.argtypes = [i64, p, p, p, p, i64, C.POINTER(C.c_double), C.POINTER(Options), C.POINTER(p)]
    L.amg_update_values.argtypes = [p, p, p, p, i64]
    L.amg_solve.argtypes = [p, p, p, d, C.POINTER(Info)]
    L.amg_free.argtypes = [p]
    L.amg_free.restype = None
    L.amg_set_precision.argtypes = [p, i32]
    L.amg_set_stream.argtypes = [p, p]
    L.amg_solve_batch.argtypes = [C.POINTER(p), C.POINTER(p), C.POINTER(p), C.POINTER(d), i32, C.POINTER(Info)]
    L.amg_solve_batch_noalloc.argtypes = [C.POINTER(p), C.POINTER(p), C.POINTER(p), C.POINTER(d), i32,
                                          C.POINTER(Info)]
    L.amg_cache_control.argtypes = [i32, i64, C.POINTER(C.c_size_t)]
    L.amg_estimate_bytes.argtypes = [i64, i64, C.POINTER(Options), C.POINTER(C.c_size_t)]
    L.amg_hierarchy_bytes.argtypes = [p, C.POINTER(C.c_size_t)]
    L.amg_num_levels.argtypes = [p, C.POINTER(i32)]
    L.amg_level_info.argtypes = [p, i32, C.POINTER(i64), C.POINTER(i32), C.POINTER(i64), C.POINTER(i32)]
    L.amg_export_level.argtypes = [p, i32, p, p, p, p, p, p, p]
    L.amg_export_level_f32.argtypes = [p, i32, p]
    L.amg_apply_precond.argtypes = [p, p, p, i32]
    L.amg_level_smooth.argtypes = [p, i32, p, p, i32, i32]
    L.amg_level_spmv.argtypes = [p, i32, p, p, i32]
    L.amg_kernel_timing_enable.argtypes = [p, C.c_char_p]
    L.amg_kernel_timing_read.argtypes = [p, C.POINTER(i64), C.POINTER(d), C.POINTER(d)]
    L.amg_engine_info.argtypes = [p, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(C.c_size_t)]
    L.amg_p1_mesh_create.argtypes = [i64, p, i64, p, p, i64, p, C.POINTER(p)]
    L.amg_p1_mesh_pattern.argtypes = [p, C.POINTER(i64), p, p]
    L.amg_p1_assemble.argtypes = [p, p, p]
    L.amg_p1_mesh_free.argtypes = [p]
    L.amg_p1_mesh_free.restype = None
    L.amg_status_string.argtypes = [i32]
    L.amg_status_string.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("amg_default_options", "amg_free", "amg_p1_mesh_free", "amg_status_string"):
            getattr(L, name).restype = i32
    _lib = L
    return L


def _check(code, what):
    if code != OK:
        raise AMGError(code, what)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def default_options() -> Options:
    o = Options()
    load().amg_default_options(C.byref(o))
    return o


def estimate_bytes(n: int, nnz: int, **opts) -> int:
    o = _options(**opts)
    b = C.c_size_t()
    _check(load().amg_estimate_bytes(n, nnz, C.byref(o), C.byref(b)), "amg_estimate_bytes")
    return b.value


def _options(precision=0, coarse_max=64, inner_iters=2, sweeps=1, outer_mmax=1, max_iters=1000, box=None,
             stream=None, engine=1, batch=1, smoother=0):
    o = default_options()
    o.precision, o.coarse_max, o.inner_iters = precision, coarse_max, inner_iters
    o.sweeps, o.outer_mmax, o.max_iters, o.engine, o.batch = sweeps, outer_mmax, max_iters, engine, batch
    o.smoother = smoother
    o._box = None
    if box is not None:
        o._box = (C.c_double * 4)(*[float(v) for v in box])
        o.box = C.cast(o._box, C.POINTER(C.c_double))
    o.stream = stream
    return o


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Hierarchy:
    """Device-resident hierarchy built by amg_setup from device tensors.

    coords: (n, 2) float64 (quadtree, amg_setup) or (n, 3) float64 (octree, amg_setup3d; box = 6 values), row_ptr:
    (n+1,) int64, col: (nnz,) int32, val: (nnz,) float64, all on one CUDA device.
    """

    def __init__(self, coords, row_ptr, col, val, box=None, precision=0, coarse_max=64, inner_iters=2, sweeps=1,
                 outer_mmax=1, max_iters=1000, stream=None, engine=1, batch=1, smoother=0, allocator=None):
        import torch
        L = load()
        if not torch.cuda.is_available():
            raise RuntimeError("quadamg needs a GPU (no HIP device visible)")
        for t, dt in ((coords, torch.float64), (row_ptr, torch.int64), (col, torch.int32), (val, torch.float64)):
            if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise TypeError("inputs must be contiguous CUDA tensors: coords f64 (n,2), row_ptr i64, col i32, "
                                "val f64")
        self.device = coords.device
        self.n = int(coords.shape[0])
        self.nnz = int(col.numel())
        self._stream = stream
        dim = int(coords.shape[1])
        if dim not in (2, 3):
            raise TypeError("coords must be (n, 2) or (n, 3)")
        self.dim = dim
        o = _options(precision, coarse_max, inner_iters, sweeps, outer_mmax, max_iters, box if dim == 2 else None,
                     _stream_handle(stream), engine, batch, smoother)
        # allocator: None = the library's pool; "torch" = torch's caching allocator; or a TorchAllocator
        if allocator == "torch":
            allocator = TorchAllocator(self.device, stream)
        self._allocator = allocator
        if allocator is not None:
            allocator.install(o)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            if dim == 3:  # the octree variant: the box (6 values) is an argument of its own
                box6 = None if box is None else (C.c_double * 6)(*[float(v) for v in box])
                _check(L.amg_setup3d(self.n, _ptr(coords), _ptr(row_ptr), _ptr(col), _ptr(val), self.nnz, box6,
                                     C.byref(o), C.byref(h)), "amg_setup3d")
            else:
                _check(L.amg_setup(self.n, _ptr(coords), _ptr(row_ptr), _ptr(col), _ptr(val), self.nnz,
                                   C.byref(o), C.byref(h)), "amg_setup")
        self._h = h
        lv = C.c_int32()
        _check(L.amg_num_levels(h, C.byref(lv)), "amg_num_levels")
        self.num_levels = lv.value

    @classmethod
    def from_problem(cls, prob, device="cuda", **kw):
        import torch
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
        kw.setdefault("box", prob.box)
        return cls(t(prob.coords, torch.float64), t(prob.row_ptr, torch.int64), t(prob.col, torch.int32),
                   t(prob.val, torch.float64), **kw)

    def close(self):
        if getattr(self, "_h", None):
            load().amg_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_values(self, row_ptr, col, val):
        """New matrix values on the pattern given to setup (same rows, same column order): amg_update_values."""
        import torch
        for t, dt in ((row_ptr, torch.int64), (col, torch.int32), (val, torch.float64)):
            if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise TypeError("inputs must be contiguous CUDA tensors: row_ptr i64, col i32, val f64")
        with torch.cuda.device(self.device):
            _check(load().amg_update_values(self._h, _ptr(row_ptr), _ptr(col), _ptr(val), int(col.numel())),
                   "amg_update_values")

    def update_problem(self, prob):
        """update_values from a host problem of the same mesh (meshgen.Problem)."""
        import torch
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=self.device)
        self.update_values(t(prob.row_ptr, torch.int64), t(prob.col, torch.int32), t(prob.val, torch.float64))

    # -- solve --------------------------------------------------------------------------------------------------
    def set_precision(self, precision: int):
        _check(load().amg_set_precision(self._h, precision), "amg_set_precision")

    def set_stream(self, stream):
        self._stream = stream
        _check(load().amg_set_stream(self._h, _stream_handle(stream)), "amg_set_stream")

    def solve(self, b, tol=1e-8, x=None, check=True):
        import torch
        if x is None:
            x = torch.empty_like(b)
        info = Info()
        code = load().amg_solve(self._h, _ptr(b), _ptr(x), float(tol), C.byref(info))
        if check and code != OK:
            raise AMGError(code, "amg_solve")
        d = info.as_dict()
        d["status"] = code    # also set when the call fails before the solve starts
        return x, d

    def apply_precond(self, r, precision=0):
        import torch
        z = torch.empty_like(r)
        _check(load().amg_apply_precond(self._h, _ptr(r), _ptr(z), precision), "amg_apply_precond")
        return z

    def smooth(self, level, f, x, forward=True, precision=0):
        x = x.clone()
        _check(load().amg_level_smooth(self._h, level, _ptr(f), _ptr(x), 1 if forward else 0, precision),
               "amg_level_smooth")
        return x

    def spmv(self, level, x, precision=0):
        import torch
        y = torch.empty_like(x)
        _check(load().amg_level_spmv(self._h, level, _ptr(x), _ptr(y), precision), "amg_level_spmv")
        return y

    # -- inspection ---------------------------------------------------------------------------------------------
    def bytes(self) -> int:
        b = C.c_size_t()
        _check(load().amg_hierarchy_bytes(self._h, C.byref(b)), "amg_hierarchy_bytes")
        return b.value

    def level_info(self, level: int) -> dict:
        n, k, ovf, L = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int32()
        _check(load().amg_level_info(self._h, level, C.byref(n), C.byref(k), C.byref(ovf), C.byref(L)),
               "amg_level_info")
        return dict(n=n.value, k=k.value, ovf_nnz=ovf.value, L=L.value)

    def export_level(self, level: int, f32: bool = False) -> dict:
        info = self.level_info(level)
        n = info["n"]
        out = dict(info)
        out["agg"] = np.empty(n, dtype=np.int32)
        out["color"] = np.empty(n, dtype=np.uint8)
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        L = load()
        if level == 0:
            _check(L.amg_export_level(self._h, 0, p(out["agg"]), p(out["color"]), None, None, None, None, None),
                   "amg_export_level")
            return out
        ns = 27 if getattr(self, "dim", 2) == 3 else 9
        out["aj"] = np.empty((n, ns), dtype=np.int32)
        out["ax"] = np.empty((n, ns), dtype=np.float64)
        out["ovf_ptr"] = np.empty(n + 1, dtype=np.int64)
        out["ovf_col"] = np.empty(info["ovf_nnz"], dtype=np.int32)
        out["ovf_val"] = np.empty(info["ovf_nnz"], dtype=np.float64)
        _check(L.amg_export_level(self._h, level, *[p(out[k]) for k in ("agg", "color", "aj", "ax", "ovf_ptr",
                                                                       "ovf_col", "ovf_val")]), "amg_export_level")
        if f32:
            out["ax32"] = np.empty((n, ns), dtype=np.float32)
            _check(L.amg_export_level_f32(self._h, level, p(out["ax32"])), "amg_export_level_f32")
        return out

    def engine_info(self, precision=0) -> dict:
        t, l, st, b = C.c_int32(), C.c_int32(), C.c_int32(), C.c_size_t()
        _check(load().amg_engine_info(self._h, precision, C.byref(t), C.byref(l), C.byref(st), C.byref(b)),
               "amg_engine_info")
        return dict(top_level=t.value, lds_level=l.value, steps=st.value, lds_bytes=b.value)

    # -- kernel timing ------------------------------------------------------------------------------------------
    def timing_enable(self, name):
        _check(load().amg_kernel_timing_enable(self._h, name.encode() if name else None), "amg_kernel_timing_enable")

    def timing_read(self):
        n, ms, b = C.c_int64(), C.c_double(), C.c_double()
        _check(load().amg_kernel_timing_read(self._h, C.byref(n), C.byref(ms), C.byref(b)), "amg_kernel_timing_read")
        return dict(launches=n.value, total_ms=ms.value, bytes_per_launch=b.value)


def cache_control(device: int = 0, limit_bytes: int = -1) -> int:
    """amg_cache_control: set the library's freed-block cache limit on `device` (limit_bytes >= 0, returning blocks
    beyond it to the driver) and return the bytes it holds."""
    out = C.c_size_t()
    _check(load().amg_cache_control(int(device), int(limit_bytes), C.byref(out)), "amg_cache_control")
    return out.value


def solve_batch(hiers, bs, xs, tols, noalloc=False):
    """amg_solve_batch (or amg_solve_batch_noalloc) over distinct hierarchies; returns (first status, list of info
    dicts)."""
    n = len(hiers)
    H = (C.c_void_p * n)(*[h._h for h in hiers])
    B = (C.c_void_p * n)(*[b.data_ptr() for b in bs])
    X = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
    T = (C.c_double * n)(*[float(t) for t in tols])
    infos = (Info * n)()
    fn = load().amg_solve_batch_noalloc if noalloc else load().amg_solve_batch
    code = fn(H, B, X, T, n, infos)
    return code, [i.as_dict() for i in infos]


class P1Mesh:
    """Device P1 assembly for a fixed triangle mesh (amg_p1_mesh_*): pattern once, values per coefficient field.

    points: (nv, 2) float64, tris: (nt, 3) int32, dof: (nv,) int32 (-1 = eliminated vertex), CUDA tensors.
    """

    def __init__(self, points, tris, dof, ndof, stream=None):
        import torch
        L = load()
        for t, dt in ((points, torch.float64), (tris, torch.int32), (dof, torch.int32)):
            if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise TypeError("inputs must be contiguous CUDA tensors: points f64 (nv,2), tris i32 (nt,3), dof i32")
        self.device = points.device
        self.nv, self.nt, self.ndof = int(points.shape[0]), int(tris.shape[0]), int(ndof)
        m = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.amg_p1_mesh_create(self.nv, _ptr(points), self.nt, _ptr(tris), _ptr(dof), self.ndof,
                                        _stream_handle(stream), C.byref(m)), "amg_p1_mesh_create")
        self._m = m
        nnz = C.c_int64()
        _check(L.amg_p1_mesh_pattern(m, C.byref(nnz), None, None), "amg_p1_mesh_pattern")
        self.nnz = nnz.value

    def pattern(self):
        """(row_ptr int64 (ndof+1,), col int32 (nnz,)) on the mesh's device."""
        import torch
        rp = torch.empty(self.ndof + 1, dtype=torch.int64, device=self.device)
        col = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        nnz = C.c_int64()
        _check(load().amg_p1_mesh_pattern(self._m, C.byref(nnz), _ptr(rp), _ptr(col)), "amg_p1_mesh_pattern")
        return rp, col

    def assemble(self, kappa=None, out=None):
        """Values (float64, (nnz,)) for per-triangle coefficients kappa (CUDA float64 (nt,), None = 1)."""
        import torch
        if out is None:
            out = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        if kappa is not None and not (kappa.is_cuda and kappa.dtype == torch.float64 and kappa.is_contiguous()
                                      and kappa.numel() == self.nt):
            raise TypeError("kappa must be a contiguous CUDA float64 tensor of one value per triangle")
        _check(load().amg_p1_assemble(self._m, None if kappa is None else _ptr(kappa), _ptr(out)), "amg_p1_assemble")
        return out

    def close(self):
        if getattr(self, "_m", None):
            load().amg_p1_mesh_free(self._m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
