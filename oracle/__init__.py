"""ctypes front end of the serial FP64 CPU oracle (``oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
benchmark's CPU-baseline leg use this module.  The GPU library never imports
it, and it imports nothing from the GPU library.
"""
import ctypes as C
import os
import subprocess

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.cpp")

STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "ENOMEM", -3: "ESINGULAR",
          -4: "EBREAKDOWN", -5: "ENAN"}


def build_lib():
    """Compile the oracle with the host compiler (always rebuilds)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", LIB_PATH + ".tmp", SRC_PATH]
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)


class _Csr(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("colind", C.c_void_p), ("val", C.c_void_p)]


class _Field(C.Structure):
    _fields_ = [("ndof", C.c_int32), ("block_size", C.c_int32), ("nns", C.c_int32),
                ("nullspace", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("order", C.c_int32), ("coarse_max", C.c_int32),
                ("max_levels", C.c_int32), ("cheb_degree", C.c_int32), ("power_its", C.c_int32),
                ("cheb_ratio", C.c_double), ("cheb_boost", C.c_double),
                ("simplec_mode", C.c_int32), ("split", C.c_void_p),
                ("schur_direct_max", C.c_int32), ("hier_fp32", C.c_int32), ("seed", C.c_uint64)]


class _SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("maxit", C.c_int32), ("flexible", C.c_int32),
                ("rtol", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32),
                ("relres", C.c_double), ("setup_s", C.c_double), ("solve_s", C.c_double),
                ("bytes", C.c_double), ("gbps", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_lib()
        L = C.CDLL(LIB_PATH)
        L.orc_setup.restype = C.c_int
        L.orc_setup.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_char_p, C.c_void_p,
                                C.POINTER(C.c_void_p)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_last_error.restype = C.c_char_p
        L.orc_precond_apply.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]
        L.orc_apply_matrix.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]
        L.orc_gmres_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                      C.c_void_p]
        for f in ("orc_hier_count",):
            getattr(L, f).argtypes = [C.c_void_p]
        L.orc_hier_nlevels.argtypes = [C.c_void_p, C.c_int]
        L.orc_hier_nfields.argtypes = [C.c_void_p, C.c_int]
        L.orc_hier_size.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.orc_hier_block_size.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.orc_hier_lambda.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.orc_hier_lambda.restype = C.c_double
        L.orc_hier_matrix.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_hier_matrix.restype = C.c_int64
        L.orc_hier_aggregates.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]
        L.orc_hier_nullspace.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]
        L.orc_node_graph.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p]
        L.orc_node_graph.restype = C.c_int64
        L.orc_mis2_aggregate.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                         C.c_void_p]
        L.orc_tentative.argtypes = [C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_power_lambda.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                                       C.c_int32]
        L.orc_power_lambda.restype = C.c_double
        L.orc_chebyshev.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                    C.c_double, C.c_double, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_int32]
        L.orc_color_nodes.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p]
        L.orc_sgs.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double,
                              C.c_int32, C.c_uint64, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                              C.c_int32, C.c_void_p]
        L.orc_splitmix64.argtypes = [C.c_uint64]
        L.orc_splitmix64.restype = C.c_uint64
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _csr_arrays(A):
    A = sp.csr_matrix(A)
    A.sort_indices()
    return (np.ascontiguousarray(A.indptr, dtype=np.int64),
            np.ascontiguousarray(A.indices, dtype=np.int32),
            np.ascontiguousarray(A.data, dtype=np.float64))


DEFAULT_OPTS = dict(sweeps=1, order="bwd", coarse_max=200, max_levels=10, cheb_degree=2,
                    power_its=10, cheb_ratio=30.0, cheb_boost=1.1, simplec_mode=0, split=None,
                    schur_direct_max=5000, hier_fp32=0, seed=0)
_ORDER = {"fwd": 0, "bwd": 1, "sym": 2}


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Oracle:
    """Serial FP64 solver context over an N x N block system."""

    def __init__(self, fields, blocks, spec, **opts):
        L = lib()
        bad = set(opts) - set(DEFAULT_OPTS)
        if bad:
            raise TypeError(f"unknown oracle options: {sorted(bad)}")
        o = dict(DEFAULT_OPTS)
        o.update(opts)
        self.sizes = [f.ndof for f in fields]
        self.n = sum(self.sizes)
        N = len(fields)
        self._keep = []
        fa = (_Field * N)()
        for i, f in enumerate(fields):
            ns = np.ascontiguousarray(f.nullspace, dtype=np.float64)
            self._keep.append(ns)
            fa[i] = _Field(f.ndof, f.block_size, ns.shape[0], _p(ns).value)
        ba = (_Csr * (N * N))()
        for i in range(N):
            for j in range(N):
                B = blocks[i][j]
                if B is None:
                    ba[i * N + j] = _Csr(self.sizes[i], self.sizes[j], 0, None, None, None)
                    continue
                p, c, v = _csr_arrays(B)
                self._keep += [p, c, v]
                ba[i * N + j] = _Csr(B.shape[0], B.shape[1], int(p[-1]), _p(p).value, _p(c).value,
                                     _p(v).value)
        split = None
        if o["split"] is not None:
            split = np.ascontiguousarray(o["split"], dtype=np.int32)
            self._keep.append(split)
        order = o["order"] if isinstance(o["order"], int) else _ORDER[o["order"]]
        self.opts = _Opts(o["sweeps"], order, o["coarse_max"], o["max_levels"], o["cheb_degree"],
                          o["power_its"], o["cheb_ratio"], o["cheb_boost"], o["simplec_mode"],
                          None if split is None else _p(split).value, o["schur_direct_max"],
                          o["hier_fp32"], o["seed"])
        h = C.c_void_p()
        rc = L.orc_setup(N, C.cast(fa, C.c_void_p), C.cast(ba, C.c_void_p), spec.encode(),
                         C.byref(self.opts), C.byref(h))
        if rc != 0:
            raise OracleError(rc, L.orc_last_error().decode())
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def _cols(self, v):
        v = np.asarray(v, dtype=np.float64)
        one = v.ndim == 1
        v = np.ascontiguousarray(v.reshape(-1, self.n))
        return v, one

    def matvec(self, x):
        x, one = self._cols(x)
        y = np.zeros_like(x)
        lib().orc_apply_matrix(self.h, _p(x), _p(y), x.shape[0])
        return y[0] if one else y

    def precond_apply(self, r):
        r, one = self._cols(r)
        z = np.zeros_like(r)
        rc = lib().orc_precond_apply(self.h, _p(r), _p(z), r.shape[0])
        if rc != 0:
            raise OracleError(rc, lib().orc_last_error().decode())
        return z[0] if one else z

    def gmres(self, b, x0=None, restart=50, maxit=1000, flexible=0, rtol=1e-8):
        b, one = self._cols(b)
        x = np.zeros_like(b) if x0 is None else np.ascontiguousarray(
            np.asarray(x0, dtype=np.float64).reshape(b.shape)).copy()
        so = _SolveOpts(restart, maxit, flexible, rtol)
        st = (_Stats * b.shape[0])()
        rc = lib().orc_gmres_solve(self.h, _p(b), _p(x), b.shape[0], C.byref(so),
                                   C.cast(st, C.c_void_p))
        if rc < 0:
            raise OracleError(rc, lib().orc_last_error().decode())
        stats = [dict(iters=s.iters, restarts=s.restarts, status=s.status, relres=s.relres,
                      setup_s=s.setup_s, solve_s=s.solve_s) for s in st]
        return (x[0] if one else x), (stats[0] if one else stats)

    # ---- hierarchy inspection ----
    def hier_count(self):
        return lib().orc_hier_count(self.h)

    def nlevels(self, h=0):
        return lib().orc_hier_nlevels(self.h, h)

    def nfields(self, h=0):
        return lib().orc_hier_nfields(self.h, h)

    def level_size(self, h, l, f=0):
        return lib().orc_hier_size(self.h, h, l, f)

    def block_size(self, h, l, f=0):
        return lib().orc_hier_block_size(self.h, h, l, f)

    def lam(self, h, l, f=0):
        return lib().orc_hier_lambda(self.h, h, l, f)

    def matrix(self, h, l, which, i=0, j=0):
        """which: 'A' (block i,j), 'P' (field i), 'R' (field i). None if absent."""
        w = {"A": 0, "P": 1, "R": 2}[which]
        L = lib()
        nr, nc = C.c_int32(), C.c_int32()
        nnz = L.orc_hier_matrix(self.h, h, l, w, i, j, None, None, None, C.byref(nr), C.byref(nc))
        if nnz < 0:
            return None
        ptr = np.zeros(nr.value + 1, np.int64)
        col = np.zeros(nnz, np.int32)
        val = np.zeros(nnz, np.float64)
        L.orc_hier_matrix(self.h, h, l, w, i, j, _p(ptr), _p(col), _p(val), None, None)
        return sp.csr_matrix((val, col, ptr), shape=(nr.value, nc.value))

    def aggregates(self, h, l, f=0):
        n = lib().orc_hier_aggregates(self.h, h, l, f, None)
        if n < 0:
            return None
        out = np.zeros(n, np.int32)
        lib().orc_hier_aggregates(self.h, h, l, f, _p(out))
        return out

    def nullspace(self, h, l, f=0):
        n = lib().orc_hier_nullspace(self.h, h, l, f, None)
        out = np.zeros(n, np.float64)
        lib().orc_hier_nullspace(self.h, h, l, f, _p(out))
        k = n // self.level_size(h, l, f)
        return out.reshape(k, -1)


# ---- building blocks ----
def node_graph(A, b):
    p, c, _ = _csr_arrays(A)
    n = A.shape[0]
    L = lib()
    nnz = L.orc_node_graph(n, b, _p(p), _p(c), None, None)
    if nnz < 0:
        raise OracleError(int(nnz), L.orc_last_error().decode())
    gp = np.zeros(n // b + 1, np.int64)
    ga = np.zeros(nnz, np.int32)
    L.orc_node_graph(n, b, _p(p), _p(c), _p(gp), _p(ga))
    return gp, ga


def mis2_aggregate(gptr, gadj, seed):
    n = len(gptr) - 1
    gptr = np.ascontiguousarray(gptr, np.int64)
    gadj = np.ascontiguousarray(gadj, np.int32)
    st = np.zeros(n, np.int32)
    agg = np.zeros(n, np.int32)
    na = lib().orc_mis2_aggregate(n, _p(gptr), _p(gadj), seed, _p(st), _p(agg))
    if na < 0:
        raise OracleError(na, lib().orc_last_error().decode())
    return st, agg, na


def tentative(agg, n_agg, b, B):
    agg = np.ascontiguousarray(agg, np.int32)
    B = np.ascontiguousarray(B, np.float64)
    k = B.shape[0]
    ndof = len(agg) * b
    ptr = np.zeros(ndof + 1, np.int64)
    col = np.zeros(ndof * k, np.int32)
    val = np.zeros(ndof * k, np.float64)
    Bc = np.zeros(k * n_agg * k, np.float64)
    ndead = lib().orc_tentative(len(agg), _p(agg), n_agg, b, k, _p(B), _p(ptr), _p(col), _p(val),
                                _p(Bc))
    P = sp.csr_matrix((val, col, ptr), shape=(ndof, n_agg * k))
    return P, Bc.reshape(k, n_agg * k), ndead


def power_lambda(A, seed=0, its=10):
    p, c, v = _csr_arrays(A)
    return lib().orc_power_lambda(A.shape[0], _p(p), _p(c), _p(v), seed, its)


def chebyshev(A, lam, b, x0=None, ratio=30.0, boost=1.1, degree=2):
    p, c, v = _csr_arrays(A)
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros_like(b) if x0 is None else np.ascontiguousarray(x0, np.float64).copy()
    rc = lib().orc_chebyshev(A.shape[0], _p(p), _p(c), _p(v), lam, ratio, boost, degree, _p(b),
                             _p(x), 1 if x0 is None else 0)
    if rc != 0:
        raise OracleError(rc, lib().orc_last_error().decode())
    return x


def color_nodes(gptr, gadj, seed):
    n = len(gptr) - 1
    gptr = np.ascontiguousarray(gptr, np.int64)
    gadj = np.ascontiguousarray(gadj, np.int32)
    col = np.zeros(n, np.int32)
    nc = lib().orc_color_nodes(n, _p(gptr), _p(gadj), seed, _p(col))
    return col, nc


def sgs(A, b, rhs, omega=1.0, steps=1, seed=0, x0=None, half=0, dd=False, sub=None):
    """Multicolour SGS from x0 (zero if None); half: forward sweeps only from
    a zero guess, backward sweeps only otherwise.  dd: the DD(GS) smoother,
    with the subdomains `sub` (node -> subdomain; None: the aggregates)."""
    p, c, v = _csr_arrays(A)
    rhs = np.ascontiguousarray(rhs, np.float64)
    x = np.zeros_like(rhs) if x0 is None else np.ascontiguousarray(x0, np.float64).copy()
    sb = None if sub is None else np.ascontiguousarray(sub, np.int32)
    rc = lib().orc_sgs(A.shape[0], _p(p), _p(c), _p(v), b, omega, steps, seed, _p(rhs), _p(x),
                       1 if x0 is None else 0, half, 1 if dd else 0, None if sb is None else _p(sb))
    if rc != 0:
        raise OracleError(rc, lib().orc_last_error().decode())
    return x


def splitmix64(x):
    return lib().orc_splitmix64(x)
