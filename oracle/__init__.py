"""CPU oracle of the Gravo MG setup + solve (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It wraps `liboracle.so`, a plain single-threaded C++
restatement of the method (see oracle.cpp for the step-to-paper map), and
shares no code with the GPU library.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")

# export codes (mirrors the enumeration in oracle.cpp)
POSITIONS, EDGE_ROWPTR, EDGE_COL, EDGE_W, SCALARS, SAMPLES, LABELS, DIST = range(8)
P_COL, P_VAL, P_CNT, TRI, A_ROWPTR, A_COL, A_VAL, COLORS, CHOL, CINV, BLOCK_COLORS = range(8, 19)

STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "INVALID_ARGUMENT", -4: "NOT_SPD", -5: "DEGENERATE"}


def build(force=True):
    """Compile liboracle.so with g++ (strict IEEE binary64, no contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", _LIB + ".tmp", _SRC]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("coarsening_ratio", ctypes.c_double),
                ("min_coarse_points", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
                ("shift_coarse_points", ctypes.c_int32), ("sample_order", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("weighting", ctypes.c_int32), ("fallback_on_vertex", ctypes.c_int32),
                ("color_passes", ctypes.c_int32), ("block_min_rows", ctypes.c_int32),
                ("autotune", ctypes.c_int32)]


def default_options(**kw):
    o = Options(ctypes.sizeof(Options), 1.0 / 8.0, 1000, 32, 2, 2, 1, 0, 0)
    o.color_passes = 3
    o.block_min_rows = 4096
    o.autotune = 1
    for k, v in kw.items():
        setattr(o, k, v)
    return o


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_build.argtypes = [ctypes.c_int64, P, ctypes.c_int64, P, P, P, P, ctypes.c_int64, P,
                                ctypes.POINTER(ctypes.c_void_p)]
        L.orc_free.argtypes = [P]
        L.orc_num_levels.argtypes = [P]
        L.orc_level_sizes.argtypes = [P, ctypes.c_int32, P]
        L.orc_export.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int64]
        L.orc_solve.argtypes = [P, P, P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_int32), P]
        L.orc_precondition.argtypes = [P, P, P, ctypes.c_int32]
        L.orc_solve_pcg.argtypes = [P, P, P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, P, P, P]
        L.orc_closest_point.argtypes = [P, P, P, P, P]
        L.orc_degenerate.argtypes = [P, P, P]
        L.orc_dsatur.argtypes = [ctypes.c_int32, P, P, P]
        L.orc_mix64.argtypes = [ctypes.c_uint64]
        L.orc_mix64.restype = ctypes.c_uint64
        if L.orc_options_size() != ctypes.sizeof(Options):
            raise RuntimeError("oracle options layout mismatch")
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status} ({STATUS.get(status, '?')})")
        self.status = status


class Hierarchy:
    """Oracle hierarchy for one geometry + system matrix."""

    def __init__(self, points, edges, indptr, indices, data, options=None):
        L = lib()
        self._keep = [np.ascontiguousarray(points, dtype=np.float64),
                      np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2),
                      np.ascontiguousarray(indptr, dtype=np.int32),
                      np.ascontiguousarray(indices, dtype=np.int32),
                      np.ascontiguousarray(data, dtype=np.float64)]
        pts, e, rp, ci, va = self._keep
        self.options = options if options is not None else default_options()
        h = ctypes.c_void_p()
        st = L.orc_build(pts.shape[0], _ptr(pts), e.shape[0], _ptr(e), _ptr(rp), _ptr(ci), _ptr(va),
                         ci.shape[0], ctypes.byref(self.options), ctypes.byref(h))
        self._keep = None
        if st != 0:
            raise OracleError(st)
        self._h = h

    @classmethod
    def from_problem(cls, prob, options=None):
        return cls(prob.points, prob.edges, prob.indptr, prob.indices, prob.data, options)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    @property
    def num_levels(self):
        return lib().orc_num_levels(self._h)

    def sizes(self, l):
        s = np.zeros(9, dtype=np.int64)
        st = lib().orc_level_sizes(self._h, l, _ptr(s))
        if st != 0:
            raise OracleError(st)
        return dict(n=int(s[0]), m=int(s[1]), nnzA=int(s[2]), nnzP=int(s[3]), colors=int(s[4]),
                    fallback=int(s[5]), samples=int(s[6]), nnzE=int(s[7]), blocks=int(s[8]))

    def export(self, l, what):
        s = self.sizes(l)
        n = s["n"]
        shape, dt = {
            POSITIONS: ((n, 3), np.float64), EDGE_ROWPTR: ((n + 1,), np.int32),
            EDGE_COL: ((s["nnzE"],), np.int32), EDGE_W: ((s["nnzE"],), np.float64),
            SCALARS: ((2,), np.float64), SAMPLES: ((s["samples"],), np.int32),
            LABELS: ((n if s["samples"] else 0,), np.int32),
            DIST: ((n if s["samples"] else 0,), np.float64),
            P_COL: ((n if s["samples"] else 0, 3), np.int32),
            P_VAL: ((n if s["samples"] else 0, 3), np.float64),
            P_CNT: ((n if s["samples"] else 0,), np.int32),
            TRI: ((n if s["samples"] else 0, 2), np.int32),
            A_ROWPTR: ((n + 1,), np.int32), A_COL: ((s["nnzA"],), np.int32),
            A_VAL: ((s["nnzA"],), np.float64),
            COLORS: ((n if s["colors"] else 0,), np.int32), CHOL: ((n, n), np.float64),
            CINV: ((n, n), np.float64), BLOCK_COLORS: ((n if s["blocks"] else 0,), np.int32),
        }[what]
        out = np.zeros(shape, dtype=dt)
        st = lib().orc_export(self._h, l, what, _ptr(out), out.nbytes)
        if st != 0:
            raise OracleError(st)
        return out

    def level(self, l):
        """All arrays of level l as a dict (missing ones are empty)."""
        d = dict(self.sizes(l))
        for name, code in [("X", POSITIONS), ("erp", EDGE_ROWPTR), ("ecol", EDGE_COL), ("ew", EDGE_W),
                           ("scalars", SCALARS), ("samples", SAMPLES), ("labels", LABELS),
                           ("dist", DIST), ("pcol", P_COL), ("pval", P_VAL), ("pcnt", P_CNT),
                           ("tri", TRI), ("arp", A_ROWPTR), ("acol", A_COL), ("aval", A_VAL),
                           ("colors", COLORS), ("block_colors", BLOCK_COLORS)]:
            d[name] = self.export(l, code)
        return d

    def chol(self):
        return self.export(self.num_levels - 1, CHOL)

    def coarse_inverse(self):
        """A_coarsest^-1 stored by columns: row k of the result is A^-1 e_k."""
        return self.export(self.num_levels - 1, CINV)

    def solve(self, b, x0=None, tol=1e-8, max_iters=100, gs_mode=0):
        """Returns (x, iterations, relative-residual history, status)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        hist = np.zeros(max_iters, dtype=np.float64)
        it = ctypes.c_int32(0)
        st = lib().orc_solve(self._h, _ptr(b), _ptr(x), tol, max_iters, gs_mode, ctypes.byref(it),
                             _ptr(hist))
        if st < 0:
            raise OracleError(st)
        return x, it.value, hist[:it.value], st


    def precondition(self, r, precision=0):
        """z = B r: one symmetric V-cycle from zero (precision 0: double, 1: float)."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros_like(r)
        st = lib().orc_precondition(self._h, _ptr(r), _ptr(z), precision)
        if st < 0:
            raise OracleError(st)
        return z

    def solve_pcg(self, b, x0=None, tol=1e-8, max_iters=100, precision=0):
        """Double-precision CG preconditioned by the symmetric V-cycle.
        Returns (x, iterations, recursive residual history, status, final true rel. residual)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        hist = np.zeros(max_iters, dtype=np.float64)
        it = ctypes.c_int32(0)
        fin = ctypes.c_double(0.0)
        st = lib().orc_solve_pcg(self._h, _ptr(b), _ptr(x), tol, max_iters, precision, ctypes.byref(it),
                                 _ptr(hist), ctypes.byref(fin))
        if st < 0:
            raise OracleError(st)
        return x, it.value, hist[:it.value], st, fin.value


def adjoint_gradients(indptr, indices, data, x, grad_x):
    """Gradients of a loss L(x) through the exact solve of A x = b (A given as CSR):
    dL/db = lambda with A^T lambda = dL/dx, and dL/dA_ij = -lambda_i x_j on A's stored
    entries.  Plain sparse direct solve (SciPy); returns (dL/db, dL/dA values in CSR order)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    n = len(indptr) - 1
    A = sp.csr_matrix((data, indices, indptr), shape=(n, n))
    lam = spla.spsolve(A.T.tocsc(), np.asarray(grad_x, dtype=np.float64))
    rows = np.repeat(np.arange(n), np.diff(indptr))
    return lam, -lam[rows] * np.asarray(x)[indices]


def closest_point(p, a, b, c):
    w = np.zeros(3)
    arr = [np.ascontiguousarray(v, dtype=np.float64) for v in (p, a, b, c)]
    region = lib().orc_closest_point(*[_ptr(v) for v in arr], _ptr(w))
    return w, region


def dsatur(rowptr, col):
    """DSATUR colouring of a graph in CSR form (the colouring of each cell of a
    level swept in block order): (colours per vertex, number of colours), or
    (None, -1) if a vertex would need 64 colours or more."""
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    m = len(rp) - 1
    out = np.zeros(max(m, 1), dtype=np.int32)
    nc = lib().orc_dsatur(m, _ptr(rp), _ptr(cl), _ptr(out))
    return (out[:m], nc) if nc >= 0 else (None, -1)


def degenerate(a, b, c):
    arr = [np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c)]
    return bool(lib().orc_degenerate(*[_ptr(v) for v in arr]))


def mix64(z):
    return int(lib().orc_mix64(int(z) & 0xFFFFFFFFFFFFFFFF))
