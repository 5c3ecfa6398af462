"""ctypes binding of libgmg.so (argument marshalling only).

The names follow include/gmg.h: gmg_build_hierarchy, gmg_solve, gmg_free,
gmg_num_levels, gmg_level_sizes, gmg_export_level.  Inputs are torch tensors
on the current HIP device; nothing here computes any part of the method, and
a missing library raises instead of falling back to anything else.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgmg.so")

STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "INVALID_ARGUMENT", -2: "OUT_OF_MEMORY",
          -3: "DEVICE_ERROR", -4: "NOT_SPD", -5: "DEGENERATE"}

# export code -> (name, dtype); sizes come from gmg_level_sizes
EXPORTS = {
    "positions": (0, np.float64), "edge_rowptr": (1, np.int32), "edge_col": (2, np.int32),
    "edge_w": (3, np.float64), "scalars": (4, np.float64), "samples": (5, np.int32),
    "labels": (6, np.int32), "dist": (7, np.float64), "p_col": (8, np.int32), "p_val": (9, np.float64),
    "p_cnt": (10, np.int32), "tri": (11, np.int32), "a_rowptr": (12, np.int32), "a_col": (13, np.int32),
    "a_val": (14, np.float64), "colors": (15, np.int32), "chol": (16, np.float64),
    "coarse_inverse": (17, np.float64), "block_colors": (18, np.int32),
}

# Symbols the library exports (checked on load).
SYMBOLS = ["gmg_default_options", "gmg_build_hierarchy", "gmg_solve", "gmg_solve_pcg", "gmg_precondition",
           "gmg_update_matrix", "gmg_pattern_outer", "gmg_solve_pcg_batched", "gmg_solve_pcg_grouped", "gmg_precondition_batched", "gmg_precondition_noalloc", "gmg_free", "gmg_status_string", "gmg_last_error",
           "gmg_num_levels", "gmg_level_sizes", "gmg_level_tuning", "gmg_export_level", "gmg_timer_start", "gmg_timer_stop"]

# gmg_precision
PRECISION = {"f64": 0, "f32": 1}

# kernel classes of gmg_timer_start
TIMER_KERNELS = {"gs_finest": 0, "residual_finest": 1, "gs_galerkin": 2}


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("coarsening_ratio", ctypes.c_double),
                ("min_coarse_points", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
                ("shift_coarse_points", ctypes.c_int32), ("sample_order", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("weighting", ctypes.c_int32), ("fallback_on_vertex", ctypes.c_int32),
                ("color_passes", ctypes.c_int32), ("block_min_rows", ctypes.c_int32),
                ("autotune", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_residual", ctypes.c_double)]


class GMGError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"gmg status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


_lib = None


def library():
    """Loads libgmg.so (built by paper_2307_04886_amd/build.py); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2307_04886_amd/build.py`")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.gmg_default_options.argtypes = [ctypes.POINTER(Options)]
    L.gmg_build_hierarchy.argtypes = [I64, P, I64, P, P, P, P, I64, ctypes.POINTER(Options), P,
                                      ctypes.POINTER(P)]
    L.gmg_solve.argtypes = [P, P, P, ctypes.c_double, I32, P, ctypes.POINTER(SolveInfo), P]
    L.gmg_solve_pcg.argtypes = [P, P, P, ctypes.c_double, I32, I32, P, ctypes.POINTER(SolveInfo), P]
    L.gmg_precondition.argtypes = [P, P, P, I32, P]
    L.gmg_update_matrix.argtypes = [P, P, P]
    L.gmg_solve_pcg_batched.argtypes = [P, I32, P, P, ctypes.c_double, I32, I32, P, ctypes.POINTER(SolveInfo)]
    L.gmg_solve_pcg_grouped.argtypes = [I32, ctypes.POINTER(P), ctypes.POINTER(I32), ctypes.POINTER(P),
                                        ctypes.POINTER(P), ctypes.c_double, I32, I32, P, ctypes.POINTER(SolveInfo),
                                        ctypes.POINTER(I32)]
    L.gmg_precondition_batched.argtypes = [P, I32, P, P, I32, P]
    L.gmg_precondition_noalloc.argtypes = [P, P, P, I32, P]
    L.gmg_pattern_outer.argtypes = [I64, P, P, P, P, ctypes.c_double, P, P]
    L.gmg_free.argtypes = [P]
    L.gmg_free.restype = None
    L.gmg_status_string.argtypes = [ctypes.c_int]
    L.gmg_status_string.restype = ctypes.c_char_p
    L.gmg_last_error.argtypes = []
    L.gmg_last_error.restype = ctypes.c_char_p
    L.gmg_num_levels.argtypes = [P, ctypes.POINTER(I32)]
    L.gmg_level_sizes.argtypes = [P, I32, P]
    L.gmg_export_level.argtypes = [P, I32, I32, P, I64]
    L.gmg_level_tuning.argtypes = [P, I32, P]
    L.gmg_timer_start.argtypes = [I32, I32]
    L.gmg_timer_stop.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64),
                                 ctypes.POINTER(ctypes.c_double)]
    _lib = L
    return L


def timer_start(kernel, expected_launches=0):
    """gmg_timer_start: time every launch of one kernel class with HIP events (measurement only)."""
    st = library().gmg_timer_start(TIMER_KERNELS[kernel], int(expected_launches))
    if st:
        raise _err(st)


def timer_stop():
    """gmg_timer_stop -> (total kernel ms, launches, algorithmic bytes)."""
    ms, n, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    st = library().gmg_timer_stop(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by))
    if st:
        raise _err(st)
    return ms.value, n.value, by.value


def default_options(**kw):
    o = Options()
    library().gmg_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _err(status):
    return GMGError(status, library().gmg_last_error().decode())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtype, shape=None, name=""):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Hierarchy:
    """A multigrid hierarchy owned by the library (gmg_build_hierarchy ... gmg_free)."""

    def __init__(self, handle, n, rowptr=None, col=None):
        self._h = handle
        self.n = n
        self.rowptr = rowptr          # A's pattern (device copies), for gradients on it
        self.col = col
        self.nnz = int(col.shape[0]) if col is not None else 0

    def __del__(self):
        self.free()

    def free(self):
        h = getattr(self, "_h", None)
        if h:
            library().gmg_free(h)
            self._h = None

    @property
    def num_levels(self):
        v = ctypes.c_int32()
        st = library().gmg_num_levels(self._h, ctypes.byref(v))
        if st:
            raise _err(st)
        return v.value

    def sizes(self, level):
        s = np.zeros(9, dtype=np.int64)
        st = library().gmg_level_sizes(self._h, level, s.ctypes.data_as(ctypes.c_void_p))
        if st:
            raise _err(st)
        return dict(n=int(s[0]), m=int(s[1]), nnzA=int(s[2]), nnzP=int(s[3]), colors=int(s[4]),
                    fallback=int(s[5]), samples=int(s[6]), nnzE=int(s[7]), blocks=int(s[8]))

    def tuning(self, level):
        """gmg_level_tuning: the row-kernel shapes of a level."""
        t = np.zeros(5, dtype=np.int32)
        st = library().gmg_level_tuning(self._h, level, t.ctypes.data_as(ctypes.c_void_p))
        if st:
            raise _err(st)
        return dict(lanes_A=int(t[0]), lanes_PT=int(t[1]), chunk=int(t[2]), block_sweep=int(t[3]),
                    uniform_width=int(t[4]))

    def export(self, level, what):
        code, dt = EXPORTS[what]
        s = self.sizes(level)
        n, has = s["n"], s["n"] if s["samples"] else 0
        count = {
            "positions": 3 * n, "edge_rowptr": n + 1, "edge_col": s["nnzE"],
            "edge_w": s["nnzE"], "scalars": 2, "samples": s["samples"], "labels": has, "dist": has,
            "p_col": 3 * has, "p_val": 3 * has, "p_cnt": has, "tri": 2 * has, "a_rowptr": n + 1,
            "a_col": s["nnzA"], "a_val": s["nnzA"], "colors": n if s["colors"] else 0, "chol": n * n,
            "coarse_inverse": n * n, "block_colors": n if s["blocks"] else 0,
        }[what]
        out = np.zeros(count, dtype=dt)
        st = library().gmg_export_level(self._h, level, code, out.ctypes.data_as(ctypes.c_void_p),
                                        out.nbytes)
        if st:
            raise _err(st)
        shapes = {"positions": (n, 3), "p_col": (has, 3), "p_val": (has, 3), "tri": (has, 2),
                  "chol": (n, n), "coarse_inverse": (n, n)}
        return out.reshape(shapes[what]) if what in shapes else out

    def solve(self, b, x=None, tol=1e-8, max_iters=100, stream=None, history=False):
        """Solves A x = b by V-cycles (in place on x if given).  Returns (x, SolveInfo, status[, hist])."""
        import torch
        pb = _dev(b, torch.float64, (self.n,), "b")
        if x is None:
            x = torch.zeros_like(b)
        px = _dev(x, torch.float64, (self.n,), "x")
        info = SolveInfo()
        hist = np.zeros(max_iters, dtype=np.float64)
        st = library().gmg_solve(self._h, pb, px, float(tol), int(max_iters), _stream_ptr(stream),
                                 ctypes.byref(info), hist.ctypes.data_as(ctypes.c_void_p))
        if st < 0:
            raise _err(st)
        if history:
            return x, info, st, hist[:info.iterations]
        return x, info, st

    def solve_pcg(self, b, x=None, tol=1e-8, max_iters=100, precision="f64", stream=None, history=False):
        """gmg_solve_pcg: double CG preconditioned by the symmetric V-cycle in `precision`
        ("f64" or "f32").  Returns (x, SolveInfo, status[, recursive residual history])."""
        import torch
        pb = _dev(b, torch.float64, (self.n,), "b")
        if x is None:
            x = torch.zeros_like(b)
        px = _dev(x, torch.float64, (self.n,), "x")
        info = SolveInfo()
        hist = np.zeros(max_iters, dtype=np.float64)
        st = library().gmg_solve_pcg(self._h, pb, px, float(tol), int(max_iters), PRECISION[precision],
                                     _stream_ptr(stream), ctypes.byref(info),
                                     hist.ctypes.data_as(ctypes.c_void_p))
        if st < 0:
            raise _err(st)
        if history:
            return x, info, st, hist[:info.iterations]
        return x, info, st

    def precondition(self, r, z=None, precision="f64", stream=None):
        """gmg_precondition: z = B r, one symmetric V-cycle from zero."""
        import torch
        pr = _dev(r, torch.float64, (self.n,), "r")
        if z is None:
            z = torch.empty_like(r)
        pz = _dev(z, torch.float64, (self.n,), "z")
        st = library().gmg_precondition(self._h, pr, pz, PRECISION[precision], _stream_ptr(stream))
        if st:
            raise _err(st)
        return z


    def precondition_noalloc(self, r, z, precision="f64", stream=None):
        """gmg_precondition_noalloc: z = B r into the caller's z, no allocation, no synchronisation."""
        import torch
        pr = _dev(r, torch.float64, (self.n,), "r")
        pz = _dev(z, torch.float64, (self.n,), "z")
        st = library().gmg_precondition_noalloc(self._h, pr, pz, PRECISION[precision], _stream_ptr(stream))
        if st:
            raise _err(st)
        return z

    def solve_pcg_batched(self, B, X=None, tol=1e-8, max_iters=100, precision="f32", stream=None):
        """gmg_solve_pcg_batched: B, X of shape (nrhs, n).  Returns (X, [SolveInfo], status)."""
        import torch
        nrhs = int(B.shape[0])
        pb = _dev(B, torch.float64, (nrhs, self.n), "B")
        if X is None:
            X = torch.zeros_like(B)
        px = _dev(X, torch.float64, (nrhs, self.n), "X")
        infos = (SolveInfo * max(nrhs, 1))()
        st = library().gmg_solve_pcg_batched(self._h, nrhs, pb, px, float(tol), int(max_iters), PRECISION[precision],
                                             _stream_ptr(stream), infos)
        if st < 0:
            raise _err(st)
        return X, list(infos)[:nrhs], st

    def precondition_batched(self, R, Z=None, precision="f32", stream=None):
        """gmg_precondition_batched: Z_q = B R_q for R of shape (nrhs, n)."""
        import torch
        nrhs = int(R.shape[0])
        pr = _dev(R, torch.float64, (nrhs, self.n), "R")
        if Z is None:
            Z = torch.empty_like(R)
        pz = _dev(Z, torch.float64, (nrhs, self.n), "Z")
        st = library().gmg_precondition_batched(self._h, nrhs, pr, pz, PRECISION[precision], _stream_ptr(stream))
        if st:
            raise _err(st)
        return Z

    def update_matrix(self, val, stream=None):
        """gmg_update_matrix: new values of A (same pattern); Galerkin operators and the
        coarsest factorisation are recomputed, the geometric hierarchy is kept."""
        import torch
        pv = _dev(val, torch.float64, (self.nnz,), "val")
        st = library().gmg_update_matrix(self._h, pv, _stream_ptr(stream))
        if st:
            raise _err(st)


def solve_pcg_grouped(hierarchies, Bs, Xs=None, tol=1e-8, max_iters=100, precision="f32", stream=None):
    """gmg_solve_pcg_grouped: one CG over many hierarchies, B_m of shape (nrhs_m <= 8, n_m).
    Returns ([X_m], [[SolveInfo]], [status_m], status)."""
    import torch
    count = len(hierarchies)
    if len(Bs) != count or (Xs is not None and len(Xs) != count):
        raise ValueError("one B (and X) per hierarchy")
    Xs = [torch.zeros_like(B) for B in Bs] if Xs is None else list(Xs)
    ph = (ctypes.c_void_p * max(count, 1))()
    pn = (ctypes.c_int32 * max(count, 1))()
    pb = (ctypes.c_void_p * max(count, 1))()
    px = (ctypes.c_void_p * max(count, 1))()
    for m, (h, B, X) in enumerate(zip(hierarchies, Bs, Xs)):
        nrhs = int(B.shape[0])
        ph[m] = h._h
        pn[m] = nrhs
        pb[m] = _dev(B, torch.float64, (nrhs, h.n), "B")
        px[m] = _dev(X, torch.float64, (nrhs, h.n), "X")
    infos = (SolveInfo * max(8 * count, 1))()
    status = (ctypes.c_int32 * max(count, 1))()
    st = library().gmg_solve_pcg_grouped(count, ph, pn, pb, px, float(tol), int(max_iters), PRECISION[precision],
                                         _stream_ptr(stream), infos, status)
    if st < 0:
        raise _err(st)
    out_infos = [list(infos[8 * m: 8 * m + int(B.shape[0])]) for m, B in enumerate(Bs)]
    return Xs, out_infos, [int(status[m]) for m in range(count)], st


def pattern_outer(rowptr, col, u, v, scale=1.0, out=None, stream=None):
    """gmg_pattern_outer: out[e] = scale * u_i * v_j on the entries (i, j) of a CSR pattern."""
    import torch
    n = int(rowptr.shape[0]) - 1
    nnz = int(col.shape[0])
    if out is None:
        out = torch.empty(nnz, dtype=torch.float64, device=u.device)
    args = [_dev(rowptr, torch.int32, (n + 1,), "rowptr"), _dev(col, torch.int32, (nnz,), "col"),
            _dev(u, torch.float64, (n,), "u"), _dev(v, torch.float64, (n,), "v")]
    po = _dev(out, torch.float64, (nnz,), "out")
    st = library().gmg_pattern_outer(n, args[0], args[1], args[2], args[3], float(scale), po, _stream_ptr(stream))
    if st:
        raise _err(st)
    return out


def build_hierarchy(points, edges, rowptr, col, val, options=None, stream=None):
    """gmg_build_hierarchy on torch tensors: points (n,3) f64, edges (m,2) int32, A as CSR
    (rowptr int32 (n+1), col int32, val f64).  All on the current HIP device."""
    import torch
    n = int(points.shape[0])
    m = int(edges.shape[0])
    nnz = int(col.shape[0])
    args = [_dev(points, torch.float64, (n, 3), "points"), _dev(edges, torch.int32, (m, 2), "edges"),
            _dev(rowptr, torch.int32, (n + 1,), "rowptr"), _dev(col, torch.int32, (nnz,), "col"),
            _dev(val, torch.float64, (nnz,), "val")]
    opt = options if options is not None else default_options()
    h = ctypes.c_void_p()
    st = library().gmg_build_hierarchy(n, args[0], m, args[1], args[2], args[3], args[4], nnz,
                                       ctypes.byref(opt), _stream_ptr(stream), ctypes.byref(h))
    if st:
        raise _err(st)
    return Hierarchy(h, n, rowptr.clone(), col.clone())


def from_problem(prob, options=None, device="cuda"):
    """Uploads a synthetic problem (numpy arrays) and builds its hierarchy."""
    import torch
    t = dict(points=torch.from_numpy(prob.points).to(device), edges=torch.from_numpy(prob.edges).to(device),
             rowptr=torch.from_numpy(prob.indptr).to(device), col=torch.from_numpy(prob.indices).to(device),
             val=torch.from_numpy(prob.data).to(device))
    return build_hierarchy(options=options, **t), t
