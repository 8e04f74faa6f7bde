"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/nfield.h declares, and rejects malformed input on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import nfgen
from paper_1605_01522_amd import nfield

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "nfield.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nfield_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = nfield.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(nfield.EXPORTS) == names


def test_default_options():
    o, _ = nfield.make_opts()
    assert (o.sweeps, o.order, o.coarse_max, o.cheb_degree, o.power_its) == (1, 1, 200, 2, 10)
    assert o.cheb_ratio == 30.0 and abs(o.cheb_boost - 1.1) < 1e-15


def test_strerror():
    assert nfield.nfield_strerror(-3) == "singular block or pivot"


def _setup_code(fields, blocks, spec):
    try:
        nfield.nfield_setup(fields, blocks, spec)
    except nfield.NFieldError as e:
        return e.code
    return 0


def test_host_validation_rejects_malformed_input():
    s = nfgen.tsi2d(nel=3)
    # unsorted columns in one row
    B = s.blocks[0][0].copy()
    B.has_sorted_indices = True
    r = 5
    a, b = B.indptr[r], B.indptr[r + 1]
    B.indices[a:b] = B.indices[a:b][::-1].copy()
    bad = [[B, s.blocks[0][1]], [s.blocks[1][0], s.blocks[1][1]]]
    # the binding sorts scipy input, so go through a raw structure
    L = nfield.lib()
    fa = (nfield.nfield_field * 2)()
    keep = []
    for i, f in enumerate(s.fields):
        ns = np.ascontiguousarray(f.nullspace)
        keep.append(ns)
        fa[i] = nfield.nfield_field(f.ndof, f.block_size, ns.shape[0], ns.ctypes.data)
    ba = (nfield.nfield_csr * 4)()
    for i in range(2):
        for j in range(2):
            M = bad[i][j]
            p = np.ascontiguousarray(M.indptr, np.int64)
            c = np.ascontiguousarray(M.indices, np.int32)
            v = np.ascontiguousarray(M.data, np.float64)
            keep += [p, c, v]
            ba[2 * i + j] = nfield.nfield_csr(M.shape[0], M.shape[1], int(p[-1]), p.ctypes.data,
                                              c.ctypes.data, v.ctypes.data)
    o, k2 = nfield.make_opts()
    h = C.c_void_p()
    rc = L.nfield_setup(2, C.cast(fa, C.c_void_p), C.cast(ba, C.c_void_p), b"BGS(AMG)",
                        C.byref(o), None, C.byref(h))
    assert rc == -1 and b"strictly increasing" in L.nfield_last_error()
    # wrong block shape
    wrong = [[s.blocks[0][0], s.blocks[0][1][:, :-1]], [s.blocks[1][0], s.blocks[1][1]]]
    assert _setup_code(s.fields, wrong, "BGS(AMG)") == -1
    # malformed specifications
    for spec in ["BGS(AMG", "FOO(AMG)", "BGS[sweeps=0](AMG)", "BGS(AMG))", "BGS[order=up](AMG)",
                 "BGS(AMG[smoother=sgs,half=2])", "BGS(AMG[smoother=sgs,omega=0])", "BGS(AMG[degree=0])",
                 "BGS(AMG[smoother=sgs,cheb_from=0])"]:
        assert _setup_code(s.fields, s.blocks, spec) == -1, spec
