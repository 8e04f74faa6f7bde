"""Python binding of libnfield.so (the C ABI declared in include/nfield.h).

Argument marshalling only: device vectors are torch tensors (float64, on the
GPU, shape (n,) or (nrhs, n) = column-major n x nrhs), the stream is torch's
current stream, and every step of the solver runs in the library's HIP
kernels.  The functions carry the C names; :class:`NField` wraps a context.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnfield.so")

STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "ENOMEM", -3: "ESINGULAR",
          -4: "EBREAKDOWN", -5: "ENAN", -6: "EHIP"}
ORDER = {"fwd": 0, "bwd": 1, "sym": 2}


class nfield_csr(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("colind", C.c_void_p), ("val", C.c_void_p)]


class nfield_field(C.Structure):
    _fields_ = [("ndof", C.c_int32), ("block_size", C.c_int32), ("nns", C.c_int32),
                ("nullspace", C.c_void_p)]


class nfield_opts(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("order", C.c_int32), ("coarse_max", C.c_int32),
                ("max_levels", C.c_int32), ("cheb_degree", C.c_int32), ("power_its", C.c_int32),
                ("cheb_ratio", C.c_double), ("cheb_boost", C.c_double),
                ("simplec_mode", C.c_int32), ("split", C.c_void_p),
                ("schur_direct_max", C.c_int32), ("hier_fp32", C.c_int32), ("seed", C.c_uint64),
                ("graphs", C.c_int32), ("block_products", C.c_int32), ("parallel_setup", C.c_int32),
                ("max_rhs", C.c_int32)]


class nfield_solve_opts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("maxit", C.c_int32), ("flexible", C.c_int32),
                ("rtol", C.c_double)]


class nfield_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32),
                ("relres", C.c_double), ("setup_s", C.c_double), ("solve_s", C.c_double),
                ("bytes", C.c_double), ("gbps", C.c_double)]


# every symbol include/nfield.h declares
EXPORTS = ["nfield_default_opts", "nfield_default_solve_opts", "nfield_setup",
           "nfield_precond_apply", "nfield_matvec", "nfield_gmres_solve", "nfield_gmres_solve_noalloc",
           "nfield_update_values", "nfield_rebuild", "nfield_prof_enable", "nfield_prof_read",
           "nfield_footprint_bytes", "nfield_precond_bytes", "nfield_size", "nfield_destroy", "nfield_strerror",
           "nfield_last_error", "nfield_hier_count", "nfield_hier_nlevels", "nfield_hier_nfields",
           "nfield_hier_size", "nfield_hier_lambda", "nfield_hier_matrix", "nfield_hier_aggregates",
           "nfield_hier_nnz", "nfield_hier_op_complexity", "nfield_hier_grid_complexity",
           "nfield_residual_history", "nfield_batch_create", "nfield_batch_submit", "nfield_batch_step",
           "nfield_batch_take", "nfield_batch_state", "nfield_batch_bytes", "nfield_batch_destroy"]

_lib = None


def lib():
    """Load libnfield.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.nfield_default_opts.argtypes = [vp]
    L.nfield_default_solve_opts.argtypes = [vp]
    L.nfield_setup.argtypes = [i32, vp, vp, C.c_char_p, vp, vp, C.POINTER(vp)]
    L.nfield_setup.restype = C.c_int
    L.nfield_precond_apply.argtypes = [vp, vp, vp, i32, vp]
    L.nfield_precond_apply.restype = C.c_int
    L.nfield_matvec.argtypes = [vp, vp, vp, i32, vp]
    L.nfield_matvec.restype = C.c_int
    L.nfield_gmres_solve.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    L.nfield_gmres_solve.restype = C.c_int
    L.nfield_gmres_solve_noalloc.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    L.nfield_gmres_solve_noalloc.restype = C.c_int
    L.nfield_update_values.argtypes = [vp, i32, i32, vp, i32, vp]
    L.nfield_update_values.restype = C.c_int
    L.nfield_rebuild.argtypes = [vp, vp]
    L.nfield_rebuild.restype = C.c_int
    L.nfield_prof_enable.argtypes = [i32]
    L.nfield_prof_read.argtypes = [i32, vp, vp, vp, vp]
    L.nfield_prof_read.restype = i32
    L.nfield_footprint_bytes.argtypes = [vp]
    L.nfield_footprint_bytes.restype = C.c_size_t
    L.nfield_precond_bytes.argtypes = [vp]
    L.nfield_precond_bytes.restype = C.c_size_t
    L.nfield_size.argtypes = [vp]
    L.nfield_size.restype = i64
    L.nfield_destroy.argtypes = [vp]
    L.nfield_strerror.argtypes = [C.c_int]
    L.nfield_strerror.restype = C.c_char_p
    L.nfield_last_error.restype = C.c_char_p
    L.nfield_hier_count.argtypes = [vp]
    for f in ("nfield_hier_nlevels", "nfield_hier_nfields"):
        getattr(L, f).argtypes = [vp, i32]
    L.nfield_hier_size.argtypes = [vp, i32, i32, i32]
    L.nfield_hier_lambda.argtypes = [vp, i32, i32, i32]
    L.nfield_hier_lambda.restype = C.c_double
    L.nfield_hier_matrix.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp]
    L.nfield_hier_matrix.restype = i64
    L.nfield_hier_aggregates.argtypes = [vp, i32, i32, i32, vp]
    L.nfield_hier_nnz.argtypes = [vp, i32, i32]
    L.nfield_hier_nnz.restype = i64
    for f in ("nfield_hier_op_complexity", "nfield_hier_grid_complexity"):
        getattr(L, f).argtypes = [vp, i32]
        getattr(L, f).restype = C.c_double
    L.nfield_residual_history.argtypes = [vp, i32, vp, i32]
    L.nfield_residual_history.restype = i32
    L.nfield_batch_create.argtypes = [vp, i32, vp, C.POINTER(vp)]
    L.nfield_batch_create.restype = C.c_int
    L.nfield_batch_submit.argtypes = [vp, i32, vp, vp, vp]
    L.nfield_batch_submit.restype = C.c_int
    L.nfield_batch_step.argtypes = [vp, vp, vp, vp, vp]
    L.nfield_batch_step.restype = C.c_int
    L.nfield_batch_take.argtypes = [vp, i32, vp, vp, vp]
    L.nfield_batch_take.restype = C.c_int
    L.nfield_batch_state.argtypes = [vp, i32]
    L.nfield_batch_state.restype = i32
    L.nfield_batch_bytes.argtypes = [vp]
    L.nfield_batch_bytes.restype = C.c_size_t
    L.nfield_batch_destroy.argtypes = [vp]
    _lib = L
    return L


class NFieldError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().nfield_last_error().decode()
        super().__init__(f"{where}: {STATUS.get(code, code)}: {msg}")
        self.code = code


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _stream(stream):
    """The stream handle to pass: the given torch stream, else torch's current
    stream (NULL, the default stream, when no GPU is visible)."""
    import torch
    if stream is None:
        if not torch.cuda.is_available():
            return C.c_void_p(None)
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t, n, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous() or t.numel() % n != 0:
        raise ValueError(f"{name} must be contiguous with a multiple of n = {n} elements")
    return C.c_void_p(t.data_ptr()), t.numel() // n


def make_opts(**kw):
    o = nfield_opts()
    lib().nfield_default_opts(C.byref(o))
    keep = []
    for k, v in kw.items():
        if k == "order" and isinstance(v, str):
            v = ORDER[v]
        if k == "split":
            if v is None:
                continue
            arr = np.ascontiguousarray(v, dtype=np.int32)
            keep.append(arr)
            v = _p(arr).value
        if not hasattr(o, k):
            raise KeyError(f"unknown option {k}")
        setattr(o, k, v)
    return o, keep


def nfield_setup(fields, blocks, spec, opts=None, stream=None):
    """fields: objects with ndof, block_size, nullspace (nns, ndof); blocks: N x N
    scipy CSR or None.  Returns a context handle (c_void_p)."""
    import scipy.sparse as sp
    L = lib()
    N = len(fields)
    keep = []
    fa = (nfield_field * N)()
    for i, f in enumerate(fields):
        ns = np.ascontiguousarray(f.nullspace, dtype=np.float64)
        keep.append(ns)
        fa[i] = nfield_field(f.ndof, f.block_size, ns.shape[0], _p(ns).value if ns.size else None)
    ba = (nfield_csr * (N * N))()
    for i in range(N):
        for j in range(N):
            B = blocks[i][j]
            if B is None:
                ba[i * N + j] = nfield_csr(fields[i].ndof, fields[j].ndof, 0, None, None, None)
                continue
            B = sp.csr_matrix(B)
            B.sort_indices()
            p = np.ascontiguousarray(B.indptr, dtype=np.int64)
            c = np.ascontiguousarray(B.indices, dtype=np.int32)
            v = np.ascontiguousarray(B.data, dtype=np.float64)
            keep += [p, c, v]
            ba[i * N + j] = nfield_csr(B.shape[0], B.shape[1], int(p[-1]), _p(p).value,
                                       _p(c).value, _p(v).value)
    if opts is None:
        opts, k2 = make_opts()
        keep += k2
    h = C.c_void_p()
    rc = L.nfield_setup(N, C.cast(fa, C.c_void_p), C.cast(ba, C.c_void_p), spec.encode(),
                        C.byref(opts), _stream(stream), C.byref(h))
    if rc != 0:
        raise NFieldError(rc, "nfield_setup")
    return h


def nfield_precond_apply(ctx, r, z, stream=None):
    n = lib().nfield_size(ctx)
    rp, k = _dev(r, n, "r")
    zp, k2 = _dev(z, n, "z")
    if k != k2:
        raise ValueError("r and z differ in shape")
    rc = lib().nfield_precond_apply(ctx, rp, zp, k, _stream(stream))
    if rc != 0:
        raise NFieldError(rc, "nfield_precond_apply")


def nfield_matvec(ctx, x, y, stream=None):
    n = lib().nfield_size(ctx)
    xp, k = _dev(x, n, "x")
    yp, k2 = _dev(y, n, "y")
    if k != k2:
        raise ValueError("x and y differ in shape")
    rc = lib().nfield_matvec(ctx, xp, yp, k, _stream(stream))
    if rc != 0:
        raise NFieldError(rc, "nfield_matvec")


def nfield_gmres_solve(ctx, b, x, restart=50, maxit=1000, flexible=0, rtol=1e-8, stream=None, noalloc=False):
    """Solves in place into x; returns (status, list of per-column stats dicts).
    noalloc: call nfield_gmres_solve_noalloc (workspace in the library's
    static scratch array, no device allocation)."""
    n = lib().nfield_size(ctx)
    bp, k = _dev(b, n, "b")
    xp, k2 = _dev(x, n, "x")
    if k != k2:
        raise ValueError("b and x differ in shape")
    so = nfield_solve_opts(restart, maxit, flexible, rtol)
    st = (nfield_stats * max(k, 1))()
    fn = lib().nfield_gmres_solve_noalloc if noalloc else lib().nfield_gmres_solve
    rc = fn(ctx, bp, xp, k, C.byref(so), C.cast(st, C.c_void_p), _stream(stream))
    if rc < 0:
        raise NFieldError(rc, "nfield_gmres_solve_noalloc" if noalloc else "nfield_gmres_solve")
    stats = [_stats_dict(s) for s in st[:k]]
    return rc, stats


def _stats_dict(s):
    return dict(iters=s.iters, restarts=s.restarts, status=s.status, relres=s.relres,
                setup_s=s.setup_s, solve_s=s.solve_s, bytes=s.bytes, gbps=s.gbps)


class Batch:
    """Iteration-level continuous batching over a context (nfield_batch_*):
    `slots` GMRES columns advanced one Arnoldi step per step(); right-hand
    sides join free slots and finished ones are taken between steps.  Holds
    a reference to its NField, and is destroyed before it."""

    def __init__(self, nf, slots, restart=50, maxit=1000, flexible=0, rtol=1e-8):
        self.nf = nf
        self.slots = slots
        so = nfield_solve_opts(restart, maxit, flexible, rtol)
        out = C.c_void_p()
        rc = lib().nfield_batch_create(nf.ctx, slots, C.byref(so), C.byref(out))
        if rc != 0:
            raise NFieldError(rc, "nfield_batch_create")
        self.b = out
        self._done = (C.c_int32 * slots)()

    def submit(self, slot, b, x0=None, stream=None):
        """b, x0: float64 CUDA tensors of n elements (copied on the stream)."""
        n = self.nf.n
        bp, k = _dev(b, n, "b")
        if k != 1:
            raise ValueError("one right-hand side per slot")
        xp = None
        if x0 is not None:
            xp, _ = _dev(x0, n, "x0")
        rc = lib().nfield_batch_submit(self.b, slot, bp, xp, _stream(stream))
        if rc != 0:
            raise NFieldError(rc, "nfield_batch_submit")

    def step(self, stream=None):
        """One step; returns (slots finished in it, slots still working)."""
        nd, na = C.c_int32(), C.c_int32()
        rc = lib().nfield_batch_step(self.b, C.cast(self._done, C.c_void_p), C.byref(nd), C.byref(na),
                                     _stream(stream))
        if rc != 0:
            raise NFieldError(rc, "nfield_batch_step")
        return [int(self._done[q]) for q in range(nd.value)], na.value

    def take(self, slot, x=None, stream=None):
        """Copy the finished slot's solution into x (float64 CUDA tensor of n
        elements, or None) and free the slot; returns its stats dict."""
        xp = None
        if x is not None:
            xp, _ = _dev(x, self.nf.n, "x")
        st = nfield_stats()
        rc = lib().nfield_batch_take(self.b, slot, xp, C.byref(st), _stream(stream))
        if rc != 0:
            raise NFieldError(rc, "nfield_batch_take")
        return _stats_dict(st)

    def state(self, slot):
        return lib().nfield_batch_state(self.b, slot)

    def nbytes(self):
        return lib().nfield_batch_bytes(self.b)

    def close(self):
        if getattr(self, "b", None):
            lib().nfield_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nfield_update_values(ctx, i, j, val, stream=None):
    """val: a float64 CUDA tensor (device copy) or a numpy array (host copy)."""
    import torch
    if isinstance(val, torch.Tensor):
        ptr, on_dev = C.c_void_p(val.data_ptr()), 1
        if not (val.is_cuda and val.dtype == torch.float64 and val.is_contiguous()):
            raise TypeError("val must be a contiguous float64 CUDA tensor")
    else:
        val = np.ascontiguousarray(val, dtype=np.float64)
        ptr, on_dev = _p(val), 0
    rc = lib().nfield_update_values(ctx, i, j, ptr, on_dev, _stream(stream))
    if rc != 0:
        raise NFieldError(rc, "nfield_update_values")


def nfield_rebuild(ctx, stream=None):
    rc = lib().nfield_rebuild(ctx, _stream(stream))
    if rc != 0:
        raise NFieldError(rc, "nfield_rebuild")


def nfield_prof_enable(on):
    lib().nfield_prof_enable(1 if on else 0)


SPMV_MODES = {0: "store", 1: "resid", 2: "add", 3: "sub", 4: "cheb", 5: "dscale", 6: "sgs",
              7: "sgs_sweep1", 8: "sgs_node", 9: "sgs_dense", 10: "ddgs", 11: "sgs_bsr"}
# kernel names as the profiler prints them (single right-hand side)
KERNEL_NAMES = {m: f"k_spmv<{{lanes}}, {m}, {{t}}>" for m in range(6)}
KERNEL_NAMES[6] = "k_sgs_color<{lanes}, {rows}, 1, {t}>"
KERNEL_NAMES[7] = "k_sgs_sweep1<{lanes}, {rows}, 1, {t}>"
KERNEL_NAMES[8] = "k_sgs_node<{lanes}, {rows}, 1, {t}>"
KERNEL_NAMES[9] = "k_dense_sweep_apply<1, {t}>"
KERNEL_NAMES[10] = "k_dd_sweep<{lanes}, {rows}, 1, {t}>"


def kernel_name(p):
    mode = [k for k, v in SPMV_MODES.items() if v == p["mode"]][0]
    t = "float" if p["fp32"] else "double"
    if (mode < 6 and p["rows"] > 0) or mode == 11:   # from a matrix's block copy: rows = block size
        if mode == 11:
            return f"k_sgs_color_bsr<{p['rows']}, {p['lanes']}, {t}>"
        return f"k_spmv_bsr<{p['rows']}, {p['lanes']}, {mode}, {t}>"
    return KERNEL_NAMES[mode].format(lanes=p["lanes"], rows=p["rows"],
                                     t="float" if p["fp32"] else "double")


def nfield_prof_read(max_keys=64):
    """Per SpMV kernel variant: dict(lanes, mode, fp32, launches, ms, bytes)."""
    key = np.zeros(max_keys, np.int32)
    cnt = np.zeros(max_keys, np.int64)
    ms = np.zeros(max_keys, np.float64)
    by = np.zeros(max_keys, np.float64)
    n = lib().nfield_prof_read(max_keys, _p(key), _p(cnt), _p(ms), _p(by))
    out = []
    for k in range(min(n, max_keys)):
        kk = int(key[k])
        lanes, rows = (kk // 1000) // 16, (kk // 1000) % 16
        out.append(dict(lanes=lanes, rows=rows, mode=SPMV_MODES[(kk // 10) % 100],
                        fp32=bool(kk % 10), launches=int(cnt[k]), ms=float(ms[k]),
                        bytes=float(by[k])))
    return out


def nfield_footprint_bytes(ctx):
    return lib().nfield_footprint_bytes(ctx)


def nfield_destroy(ctx):
    lib().nfield_destroy(ctx)


def nfield_strerror(code):
    return lib().nfield_strerror(code).decode()


class NField:
    """A solver context for one block system (owns the device hierarchy)."""

    def __init__(self, fields, blocks, spec, stream=None, **opts):
        o, keep = make_opts(**opts)
        self._keep = keep
        self.ctx = nfield_setup(fields, blocks, spec, o, stream)
        self.n = lib().nfield_size(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            nfield_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def precond_apply(self, r, z=None, stream=None):
        import torch
        z = torch.empty_like(r) if z is None else z
        nfield_precond_apply(self.ctx, r, z, stream)
        return z

    def matvec(self, x, y=None, stream=None):
        import torch
        y = torch.empty_like(x) if y is None else y
        nfield_matvec(self.ctx, x, y, stream)
        return y

    def gmres_solve(self, b, x=None, stream=None, **kw):
        import torch
        x = torch.zeros_like(b) if x is None else x
        rc, stats = nfield_gmres_solve(self.ctx, b, x, stream=stream, **kw)
        return x, stats

    def footprint_bytes(self):
        return nfield_footprint_bytes(self.ctx)

    def precond_bytes(self):
        return lib().nfield_precond_bytes(self.ctx)

    def update_values(self, i, j, val, stream=None):
        nfield_update_values(self.ctx, i, j, val, stream)

    def rebuild(self, stream=None):
        nfield_rebuild(self.ctx, stream)

    # ---- hierarchy inspection (host copies) ----
    def hier_count(self):
        return lib().nfield_hier_count(self.ctx)

    def nlevels(self, h=0):
        return lib().nfield_hier_nlevels(self.ctx, h)

    def nfields(self, h=0):
        return lib().nfield_hier_nfields(self.ctx, h)

    def level_size(self, h, l, f=0):
        return lib().nfield_hier_size(self.ctx, h, l, f)

    def lam(self, h, l, f=0):
        return lib().nfield_hier_lambda(self.ctx, h, l, f)

    def matrix(self, h, l, which, i=0, j=0):
        import scipy.sparse as sp
        w = {"A": 0, "P": 1, "R": 2}[which]
        nr, nc = C.c_int32(), C.c_int32()
        L = lib()
        nnz = L.nfield_hier_matrix(self.ctx, h, l, w, i, j, None, None, None, C.byref(nr),
                                   C.byref(nc))
        if nnz == -1:
            return None
        if nnz < 0:
            raise NFieldError(-6, "nfield_hier_matrix")
        ptr = np.zeros(nr.value + 1, np.int64)
        col = np.zeros(max(nnz, 1), np.int32)
        val = np.zeros(max(nnz, 1), np.float64)
        L.nfield_hier_matrix(self.ctx, h, l, w, i, j, _p(ptr), _p(col), _p(val), None, None)
        return sp.csr_matrix((val[:nnz], col[:nnz], ptr), shape=(nr.value, nc.value))

    def level_nnz(self, h, l):
        return lib().nfield_hier_nnz(self.ctx, h, l)

    def complexity(self, h=0):
        """(operator complexity, grid complexity) of hierarchy h."""
        L = lib()
        return L.nfield_hier_op_complexity(self.ctx, h), L.nfield_hier_grid_complexity(self.ctx, h)

    def residual_history(self, col=0):
        """Relative residual estimates after every Arnoldi step of the last
        solve, for one column (None if the last solve had no such column)."""
        L = lib()
        n = L.nfield_residual_history(self.ctx, col, None, 0)
        if n < 0:
            return None
        out = np.zeros(max(n, 1), np.float64)
        L.nfield_residual_history(self.ctx, col, _p(out), n)
        return out[:n]

    def aggregates(self, h, l, f=0):
        L = lib()
        n = L.nfield_hier_aggregates(self.ctx, h, l, f, None)
        if n < 0:
            return None
        out = np.zeros(n, np.int32)
        L.nfield_hier_aggregates(self.ctx, h, l, f, _p(out))
        return out
