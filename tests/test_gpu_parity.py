"""GPU library (through the C ABI) against the CPU oracle, on the same seeded
inputs.

Bars: aggregates bit-exact; hierarchy patterns identical and values within
1e-12 relative; SpMV within 1e-12 of |A||x| per entry; solutions within 1e-6
relative of the oracle at rtol 1e-8 with a true residual below 1e-8.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import nfgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1605_01522_amd import nfield
    nfield.lib()
    return torch.device("cuda:0")


def _gpu(s, spec, **opts):
    from paper_1605_01522_amd import NField
    return NField(s.fields, s.blocks, spec, **opts)


TSI_OPTS = dict(sweeps=2, order="bwd")


# ------------------------------------------------------------------- SpMV
@pytest.mark.parametrize("nel", [3, 17, 32])
def test_block_spmv_parity(dev, nel):
    _say(f"case spmv nel={nel}")
    s = nfgen.tsi2d(nel=nel, seed=nel)
    g = _gpu(s, "BGS(LU)" if nel <= 3 else "BGS(AMG)", **TSI_OPTS)
    x = np.random.default_rng(nel).standard_normal((2, s.n))
    y = g.matvec(torch.tensor(x, device=dev)).cpu().numpy()
    A = s.assembled()
    ref = np.stack([A @ xi for xi in x])
    bound = 1e-12 * np.stack([abs(A) @ abs(xi) for xi in x])
    assert np.all(np.abs(y - ref) <= bound)


# ------------------------------------------------------------- hierarchy
def _compare_hierarchies(g, o):
    assert g.hier_count() == o.hier_count()
    for h in range(o.hier_count()):
        assert g.nlevels(h) == o.nlevels(h), (h, g.nlevels(h), o.nlevels(h))
        nf_ = o.nfields(h)
        for l in range(o.nlevels(h)):
            for f in range(nf_):
                assert g.level_size(h, l, f) == o.level_size(h, l, f)
                ag, ao = g.aggregates(h, l, f), o.aggregates(h, l, f)
                if ao is None:
                    assert ag is None
                else:
                    assert np.array_equal(ag, ao), (h, l, f)          # bit-exact
                lo, lg = o.lam(h, l, f), g.lam(h, l, f)
                if l + 1 < o.nlevels(h):
                    assert abs(lg - lo) <= 1e-12 * abs(lo), (h, l, f, lg, lo)
            for which, pairs in (("A", [(i, j) for i in range(nf_) for j in range(nf_)]),
                                 ("P", [(i, 0) for i in range(nf_)]),
                                 ("R", [(i, 0) for i in range(nf_)])):
                for i, j in pairs:
                    Mo = o.matrix(h, l, which, i, j)
                    Mg = g.matrix(h, l, which, i, j)
                    if Mo is None:
                        assert Mg is None
                        continue
                    assert np.array_equal(Mg.indptr, Mo.indptr), (h, l, which, i, j)
                    assert np.array_equal(Mg.indices, Mo.indices), (h, l, which, i, j)
                    scale = max(np.abs(Mo.data).max(), 1e-300)
                    assert np.abs(Mg.data - Mo.data).max() <= 1e-12 * scale, (h, l, which, i, j)


@pytest.mark.parametrize("nel,coarse_max,seed", [(8, 20, 0), (20, 50, 3), (32, 200, 0)])
def test_bgs_amg_hierarchy_parity(dev, nel, coarse_max, seed):
    _say(f"case hierarchy BGS(AMG) nel={nel} coarse_max={coarse_max} seed={seed}")
    s = nfgen.tsi2d(nel=nel, seed=seed)
    o = oracle.Oracle(s.fields, s.blocks, "BGS(AMG)", coarse_max=coarse_max, seed=seed, **TSI_OPTS)
    g = _gpu(s, "BGS(AMG)", coarse_max=coarse_max, seed=seed, **TSI_OPTS)
    _compare_hierarchies(g, o)


def test_mono_amg_hierarchy_parity(dev):
    _say("case hierarchy AMG(BGS) nel=24")
    s = nfgen.tsi2d(nel=24, seed=2)
    o = oracle.Oracle(s.fields, s.blocks, "AMG(BGS)", coarse_max=80, **TSI_OPTS)
    g = _gpu(s, "AMG(BGS)", coarse_max=80, **TSI_OPTS)
    _compare_hierarchies(g, o)


# ----------------------------------------------------- preconditioner apply
SPECS = ["BGS(AMG)", "BGS[order=fwd](AMG)", "BGS[sweeps=3,order=sym](AMG)", "BGS(LU)",
         "SIMPLE(AMG;AMG)", "SIMPLE(AMG;LU)", "AMG(BGS)", "AMG(BGS[order=fwd])",
         "BGS(AMG[smoother=sgs,omega=0.8])", "BGS(AMG[smoother=sgs,omega=1.1,steps=2])",
         "AMG[smoother=sgs,omega=0.9](BGS)", "BGS(AMG[degree=3])",
         "BGS(AMG[smoother=sgs,omega=0.9,half=1])", "AMG[smoother=sgs,omega=0.9,half=1](BGS)",
         "BGS(AMG[smoother=sgs,omega=0.8,half=1,steps=2])",
         "BGS(AMG[smoother=ddgs,omega=0.79,ddmin=1])", "BGS(AMG[smoother=ddgs,omega=0.9,half=1,ddmin=1])",
         "AMG[smoother=ddgs,omega=0.8,ddmin=1](BGS)", "BGS(AMG[smoother=ddgs,omega=1.1,half=1,steps=2,ddmin=1])",
         "BGS(AMG[smoother=ddgs,omega=0.9,half=1])", "BGS(DDGS[omega=0.79,ddmin=1])",
         "BGS[sweeps=1](DDGS[omega=0.69,steps=2,ddmin=1])"]


@pytest.mark.parametrize("spec", SPECS)
def test_precond_apply_parity(dev, spec):
    _say(f"case precond {spec}")
    nel = 10 if "LU" in spec and "SIMPLE" not in spec else 20
    s = nfgen.tsi2d(nel=nel, seed=4)
    opts = dict(coarse_max=40, **TSI_OPTS)
    o = oracle.Oracle(s.fields, s.blocks, spec, **opts)
    g = _gpu(s, spec, **opts)
    r = np.random.default_rng(7).standard_normal((3, s.n))
    zo = o.precond_apply(r)
    zg = g.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    for k in range(3):
        assert np.linalg.norm(zg[k] - zo[k]) <= 1e-10 * np.linalg.norm(zo[k]), (spec, k)


# ------------------------------------------------------------ end to end
@pytest.mark.parametrize("nel,seed,spec", [(32, 0, "BGS(AMG)"), (32, 1, "BGS(AMG)"), (13, 2, "BGS(AMG)"),
                                           (32, 0, "AMG(BGS)"), (32, 0, "SIMPLE(AMG;AMG)"),
                                           (32, 0, "BGS(DDGS[omega=0.79,ddmin=1])")])
def test_gmres_solution_parity(dev, nel, seed, spec):
    _say(f"case gmres {spec} nel={nel} seed={seed}")
    s = nfgen.tsi2d(nel=nel, seed=seed, nrhs=2)
    o = oracle.Oracle(s.fields, s.blocks, spec, seed=seed, **TSI_OPTS)
    g = _gpu(s, spec, seed=seed, **TSI_OPTS)
    A = s.assembled()
    x, st = g.gmres_solve(torch.tensor(s.rhs, device=dev), rtol=1e-8)
    x = x.cpu().numpy()
    for k in range(2):
        xo, so = o.gmres(s.rhs[k], rtol=1e-8)
        res = np.linalg.norm(s.rhs[k] - A @ x[k]) / np.linalg.norm(s.rhs[k])
        assert st[k]["status"] == 0 and res < 1e-8
        assert abs(st[k]["relres"] - res) < 1e-10
        assert np.linalg.norm(x[k] - xo) <= 1e-6 * np.linalg.norm(xo)
        assert abs(st[k]["iters"] - so["iters"]) <= 2, (st[k]["iters"], so["iters"])


def test_flexible_and_restart(dev):
    _say("case gmres flexible / short restart")
    s = nfgen.tsi2d(nel=24, seed=5)
    g = _gpu(s, "BGS(AMG)", **TSI_OPTS)
    A = s.assembled()
    b = torch.tensor(s.rhs[0], device=dev)
    for restart, flexible in [(50, 1), (5, 0), (4, 1)]:
        x, st = g.gmres_solve(b, restart=restart, flexible=flexible, rtol=1e-9)
        xr = x.cpu().numpy()
        res = np.linalg.norm(s.rhs[0] - A @ xr) / np.linalg.norm(s.rhs[0])
        assert st[0]["status"] == 0 and res < 1e-9, (restart, flexible, res)


def test_precision_form_fp32_hierarchy(dev):
    _say("case precision form")
    s = nfgen.tsi2d(nel=32, seed=0)
    o = oracle.Oracle(s.fields, s.blocks, "BGS(AMG)", **TSI_OPTS)
    g = _gpu(s, "BGS(AMG)", hier_fp32=1, **TSI_OPTS)
    A = s.assembled()
    x, st = g.gmres_solve(torch.tensor(s.rhs[0], device=dev), flexible=1, rtol=1e-8)
    x = x.cpu().numpy()
    xo, so = o.gmres(s.rhs[0], rtol=1e-8)
    res = np.linalg.norm(s.rhs[0] - A @ x) / np.linalg.norm(s.rhs[0])
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    _say(f"precision form: iters {st[0]['iters']} (fp64 oracle {so['iters']}), relres {res:.2e}, err {err:.2e}")
    assert st[0]["status"] == 0 and res < 1e-8 and err < 1e-6


@pytest.mark.parametrize("nel", [16, 64])
def test_serving_configuration_parity(dev, nel):
    """The configuration the serving form runs (BGS(AMG), two backward
    sweeps, Chebyshev over [lambda/8, 1.1 lambda]) against the oracle: the
    FP64 preconditioner application, and the FP32-hierarchy flexible solve
    the server uses against the FP64 oracle solution."""
    from bench import SERVE_OPTS, SERVE_SPEC
    _say(f"case serving configuration nel={nel}")
    s = nfgen.tsi2d(nel=nel, seed=0)
    o = oracle.Oracle(s.fields, s.blocks, SERVE_SPEC, **SERVE_OPTS)
    g = _gpu(s, SERVE_SPEC, **SERVE_OPTS)
    r = np.random.default_rng(5).standard_normal(s.n)
    zo = o.precond_apply(r)
    zg = g.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    assert np.linalg.norm(zg - zo) <= 1e-10 * np.linalg.norm(zo)
    g32 = _gpu(s, SERVE_SPEC, hier_fp32=1, **SERVE_OPTS)
    x, st = g32.gmres_solve(torch.tensor(s.rhs[0], device=dev), flexible=1, rtol=1e-8)
    x = x.cpu().numpy()
    xo, so = o.gmres(s.rhs[0], rtol=1e-8)
    res = np.linalg.norm(s.rhs[0] - s.assembled() @ x) / np.linalg.norm(s.rhs[0])
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    _say(f"  fp32 hierarchy iters {st[0]['iters']} (fp64 oracle {so['iters']}), relres {res:.2e}, err {err:.2e}")
    assert st[0]["status"] == 0 and res < 1e-8 and err < 1e-6


def test_sgs_block_copy_parity(dev):
    """A level of at least 4,096 nodes made of dense 2 x 2 blocks (the
    plane-strain field on a 64 x 64 grid) relaxes from its block copy for one
    right-hand side: the preconditioner is the oracle's, and the block kernel
    is the one that ran; several right-hand sides take the CSR kernel."""
    from paper_1605_01522_amd import nfield
    _say("case Gauss-Seidel from the block copy")
    s = nfgen.tsi2d(nel=64, seed=1)
    spec = "BGS(AMG[smoother=sgs,omega=0.9])"
    opts = dict(coarse_max=200, **TSI_OPTS)
    o = oracle.Oracle(s.fields, s.blocks, spec, **opts)
    g = _gpu(s, spec, **opts)
    r = np.random.default_rng(3).standard_normal((2, s.n))
    nfield.nfield_prof_enable(1)
    z1 = g.precond_apply(torch.tensor(r[0], device=dev)).cpu().numpy()
    torch.cuda.synchronize()
    prof = nfield.nfield_prof_read()
    nfield.nfield_prof_enable(0)
    assert any(p["mode"] == "sgs_bsr" for p in prof), [p["mode"] for p in prof]
    z2 = g.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    zo = o.precond_apply(r)
    assert np.linalg.norm(z1 - zo[0]) <= 1e-10 * np.linalg.norm(zo[0])
    for k in range(2):
        assert np.linalg.norm(z2[k] - zo[k]) <= 1e-10 * np.linalg.norm(zo[k])
    x, st = g.gmres_solve(torch.tensor(s.rhs[0], device=dev), rtol=1e-8)
    xo, so = o.gmres(s.rhs[0], rtol=1e-8)
    x = x.cpu().numpy()
    assert st[0]["status"] == 0 and np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)
    assert abs(st[0]["iters"] - so["iters"]) <= 2


def test_sgs_block_copy_fp32_precision_form(dev):
    """The same level in the precision form: its FP32 block copy relaxes one
    right-hand side (the kernel that ran is the FP32 block kernel), and
    flexible GMRES around the FP32 hierarchy reaches the FP64 oracle's
    solution."""
    from paper_1605_01522_amd import nfield
    _say("case Gauss-Seidel from an FP32 block copy (precision form)")
    s = nfgen.tsi2d(nel=64, seed=1)
    spec = "BGS(AMG[smoother=sgs,omega=0.9])"
    opts = dict(coarse_max=200, **TSI_OPTS)
    o = oracle.Oracle(s.fields, s.blocks, spec, **opts)
    g = _gpu(s, spec, hier_fp32=1, **opts)
    nfield.nfield_prof_enable(1)
    x, st = g.gmres_solve(torch.tensor(s.rhs[0], device=dev), flexible=1, rtol=1e-8)
    torch.cuda.synchronize()
    prof = nfield.nfield_prof_read()
    nfield.nfield_prof_enable(0)
    assert any(p["mode"] == "sgs_bsr" and p["fp32"] for p in prof), [(p["mode"], p["fp32"]) for p in prof]
    x = x.cpu().numpy()
    xo, so = o.gmres(s.rhs[0], rtol=1e-8)
    res = np.linalg.norm(s.rhs[0] - s.assembled() @ x) / np.linalg.norm(s.rhs[0])
    _say(f"  fp32 block copy: iters {st[0]['iters']} (fp64 oracle {so['iters']}), relres {res:.2e}")
    assert st[0]["status"] == 0 and res < 1e-8
    assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)


# ------------------------------------------------------------ edge cases
def test_single_level_is_exact(dev):
    _say("case single level")
    s = nfgen.tsi2d(nel=4)
    g = _gpu(s, "BGS[sweeps=1,order=fwd](AMG)", coarse_max=1000)
    assert [g.nlevels(h) for h in range(g.hier_count())] == [1, 1]
    r = np.random.default_rng(0).standard_normal(s.n)
    z = g.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    n0 = s.fields[0].ndof
    z0 = np.linalg.solve(s.blocks[0][0].toarray(), r[:n0])
    z1 = np.linalg.solve(s.blocks[1][1].toarray(), r[n0:] - s.blocks[1][0] @ z0)
    assert np.allclose(z, np.concatenate([z0, z1]), rtol=1e-10, atol=1e-12)


def test_zero_nan_and_maxit(dev):
    _say("case zero / nan / maxit")
    from paper_1605_01522_amd import nfield
    s = nfgen.tsi2d(nel=6)
    g = _gpu(s, "BGS(AMG)", coarse_max=20)
    x, st = g.gmres_solve(torch.zeros(s.n, dtype=torch.float64, device=dev))
    assert st[0]["iters"] == 0 and st[0]["status"] == 0 and float(x.abs().max()) == 0.0
    b = torch.tensor(s.rhs[0], device=dev)
    b[3] = float("nan")
    with pytest.raises(nfield.NFieldError) as e:
        g.gmres_solve(b)
    assert e.value.code == -5
    x, st = g.gmres_solve(torch.tensor(s.rhs[0], device=dev), maxit=1, rtol=1e-14)
    assert st[0]["status"] == 1 and st[0]["iters"] == 1


def test_singular_inputs(dev):
    _say("case singular inputs")
    from paper_1605_01522_amd import nfield
    s = nfgen.tsi2d(nel=4)
    bad = [[s.blocks[0][0], s.blocks[0][1]], [s.blocks[1][0], None]]
    with pytest.raises(nfield.NFieldError) as e:
        _gpu(nfgen.BlockSystem(s.fields, bad, s.rhs), "BGS(AMG)")
    assert e.value.code == -3


# ------------------------------------------------- 3-field FSI-like system
# the benchmarked configuration, and the ones it was tuned from
FSI_SPEC = "SIMPLE(BGS(AMG[degree=1]);AMG[smoother=sgs,omega=0.69,half=1,steps=2])"
FSI_SPEC_H1 = "SIMPLE(BGS(AMG[degree=1]);AMG[smoother=sgs,omega=0.85,half=1])"
FSI_SPEC_FULL = "SIMPLE(BGS(AMG[degree=1]);AMG[smoother=sgs,omega=0.65])"
FSI_SPEC_D2 = "SIMPLE(BGS(AMG);AMG[smoother=sgs,omega=0.69])"
FSI_OPTS = dict(split=[0, 0, 1], simplec_mode=2, coarse_max=2000, cheb_ratio=4.0)
FSI_OPTS_ABS = dict(split=[0, 0, 1])
# the paper's own smoother on the fluid (DD(GS), subdomains = aggregates)
FSI_SPEC_DD = "SIMPLE(BGS(AMG[degree=1]);AMG[smoother=ddgs,omega=0.69,half=1,steps=2,ddmin=1])"
# Petrov-Galerkin transfers on the fluid (Sec. 7: PG-AMG for the fluid)
FSI_SPEC_PG = "SIMPLE(BGS(AMG[degree=1]);AMG[smoother=sgs,omega=0.69,half=1,steps=2,pg=1])"


@pytest.mark.parametrize("n,layers,spec,opts", [(6, 2, FSI_SPEC, FSI_OPTS), (6, 2, FSI_SPEC_H1, FSI_OPTS),
                                                (6, 2, FSI_SPEC_FULL, FSI_OPTS),
                                                (6, 2, FSI_SPEC_D2, FSI_OPTS_ABS), (12, 3, FSI_SPEC, FSI_OPTS),
                                                (12, 3, FSI_SPEC_DD, FSI_OPTS), (16, 4, FSI_SPEC_DD, FSI_OPTS),
                                                (12, 3, FSI_SPEC_PG, FSI_OPTS), (16, 4, FSI_SPEC_PG, FSI_OPTS)])
def test_fsi_hierarchy_precond_and_solution_parity(dev, n, layers, spec, opts):
    _say(f"case fsi3d n={n} layers={layers} {spec} {opts}")
    s = nfgen.fsi3d(n=n, layers=layers, seed=n)
    o = oracle.Oracle(s.fields, s.blocks, spec, **opts)
    g = _gpu(s, spec, **opts)
    _compare_hierarchies(g, o)
    r = np.random.default_rng(n).standard_normal((2, s.n))
    zo = o.precond_apply(r)
    zg = g.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    for k in range(2):
        assert np.linalg.norm(zg[k] - zo[k]) <= 1e-10 * np.linalg.norm(zo[k])
    A = s.assembled()
    x, st = g.gmres_solve(torch.tensor(s.rhs[0], device=dev), rtol=1e-8, maxit=1000)
    x = x.cpu().numpy()
    xo, so = o.gmres(s.rhs[0], rtol=1e-8, maxit=1000)
    res = np.linalg.norm(s.rhs[0] - A @ x) / np.linalg.norm(s.rhs[0])
    assert st[0]["status"] == 0 and res < 1e-8
    assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)
    assert abs(st[0]["iters"] - so["iters"]) <= 2, (st[0]["iters"], so["iters"])


@pytest.fixture(scope="module")
def fsi_full():
    s = nfgen.fsi3d(n=40, layers=8, seed=0)
    return s


def test_fsi_full_size_sampled_parity(dev, fsi_full):
    """The benchmarked 0.49M-dof system: SpMV rows sampled one by one, every
    aggregate of the finest level of every hierarchy bit-exact, one
    preconditioner application against the oracle, and the solve's true
    residual."""
    _say("case fsi3d full size (n=40, layers=8)")
    s = fsi_full
    g = _gpu(s, FSI_SPEC, **FSI_OPTS)
    A = s.assembled()
    rng = np.random.default_rng(11)
    xv = rng.standard_normal(s.n)
    y = g.matvec(torch.tensor(xv, device=dev)).cpu().numpy()
    rows = rng.choice(s.n, 2000, replace=False)
    for r in rows:
        lo, hi = A.indptr[r], A.indptr[r + 1]
        ref = float(np.dot(A.data[lo:hi], xv[A.indices[lo:hi]]))
        bound = 1e-12 * float(np.dot(np.abs(A.data[lo:hi]), np.abs(xv[A.indices[lo:hi]])))
        assert abs(y[r] - ref) <= bound, r
    o = oracle.Oracle(s.fields, s.blocks, FSI_SPEC, **FSI_OPTS)
    assert g.hier_count() == o.hier_count()
    for h in range(o.hier_count()):
        assert g.nlevels(h) == o.nlevels(h)
        assert np.array_equal(g.aggregates(h, 0), o.aggregates(h, 0)), h
        for l in range(o.nlevels(h)):
            assert g.level_size(h, l) == o.level_size(h, l)
    r = rng.standard_normal(s.n)
    zo = o.precond_apply(r)
    zg = g.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    assert np.linalg.norm(zg - zo) <= 1e-9 * np.linalg.norm(zo)
    x, st = g.gmres_solve(torch.tensor(s.rhs[0], device=dev), rtol=1e-8, maxit=1000)
    x = x.cpu().numpy()
    res = np.linalg.norm(s.rhs[0] - A @ x) / np.linalg.norm(s.rhs[0])
    _say(f"full-size fsi3d: iters {st[0]['iters']} relres {res:.2e}")
    assert st[0]["status"] == 0 and res < 1e-8
    # the whole solve against the oracle's solve of the same system
    xo, so = o.gmres(s.rhs[0], rtol=1e-8, maxit=1000)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    _say(f"full-size fsi3d: oracle iters {so['iters']}, relative difference {err:.2e}")
    assert so["status"] == 0
    assert err <= 1e-6
    assert abs(st[0]["iters"] - so["iters"]) <= 2, (st[0]["iters"], so["iters"])


# ------------------------------------------ Petrov-Galerkin transfers
@pytest.mark.parametrize("n,spec", [(10, "AMG[smoother=sgs,omega=0.85,half=1,pg=1]"), (14, "AMG[smoother=sgs,omega=0.85,half=1,pg=1]")])
def test_pg_hierarchy_parity(dev, n, spec):
    """Petrov-Galerkin hierarchy of the nonsymmetric fluid block: P, R (from
    A^T) and R A P against the oracle's, preconditioner and solution."""
    _say(f"case Petrov-Galerkin {spec} n={n}")
    s = nfgen.fsi3d(n=n, layers=2, seed=3)
    sub = nfgen.BlockSystem([s.fields[2]], [[s.blocks[2][2]]], s.rhs[:, s.offsets()[2]:])
    o = oracle.Oracle(sub.fields, sub.blocks, spec, coarse_max=100)
    g = _gpu(sub, spec, coarse_max=100)
    _compare_hierarchies(g, o)
    r = np.random.default_rng(14).standard_normal(sub.n)
    zo = o.precond_apply(r)
    zg = g.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    assert np.linalg.norm(zg - zo) <= 1e-10 * np.linalg.norm(zo)
    A = sub.assembled()
    x, st = g.gmres_solve(torch.tensor(sub.rhs[0], device=dev), rtol=1e-8, maxit=500)
    xo, so = o.gmres(sub.rhs[0], rtol=1e-8, maxit=500)
    x = x.cpu().numpy()
    assert st[0]["status"] == 0 and so["status"] == 0
    assert np.linalg.norm(sub.rhs[0] - A @ x) < 1e-8 * np.linalg.norm(sub.rhs[0])
    assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)
    assert abs(st[0]["iters"] - so["iters"]) <= 2


# --------------------------------------- SIMPLEC literal diagonal |sum_j a_ij|
@pytest.mark.parametrize("spec", ["SIMPLE(AMG;AMG)", "SIMPLE(LU;LU)"])
def test_simplec_literal_row_sums_parity(dev, spec):
    """SIMPLE with the literal SIMPLEC diagonal (simplec_mode=1) on the
    heat-first TSI-like system, whose predictor rows have nonzero sums:
    preconditioner application and solution against the oracle."""
    _say(f"case SIMPLEC literal {spec}")
    s = nfgen.permute_fields(nfgen.tsi2d(nel=20, seed=6, nrhs=2), [1, 0])
    opts = dict(simplec_mode=1, coarse_max=40)
    o = oracle.Oracle(s.fields, s.blocks, spec, **opts)
    g = _gpu(s, spec, **opts)
    r = np.random.default_rng(9).standard_normal((2, s.n))
    zo = o.precond_apply(r)
    zg = g.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    for k in range(2):
        assert np.linalg.norm(zg[k] - zo[k]) <= 1e-10 * np.linalg.norm(zo[k]), k
    A = s.assembled()
    x, st = g.gmres_solve(torch.tensor(s.rhs, device=dev), rtol=1e-8)
    x = x.cpu().numpy()
    for k in range(2):
        xo, so = o.gmres(s.rhs[k], rtol=1e-8)
        res = np.linalg.norm(s.rhs[k] - A @ x[k]) / np.linalg.norm(s.rhs[k])
        assert st[k]["status"] == 0 and res < 1e-8
        assert np.linalg.norm(x[k] - xo) <= 1e-6 * np.linalg.norm(xo)
        assert abs(st[k]["iters"] - so["iters"]) <= 2


# ------------------------------------------- nonsymmetric block patterns
@pytest.mark.parametrize("spec", ["BGS(AMG[smoother=sgs,omega=0.9])", "BGS(AMG)",
                                  "AMG[smoother=sgs,omega=0.9,half=1](BGS)"])
def test_one_sided_pattern_parity(dev, spec):
    """Diagonal blocks whose patterns are not symmetric (row u couples to v,
    row v not to u): the node graphs are the symmetric union on both sides,
    so aggregates are bit-exact and the colourings keep every coupled pair
    apart; hierarchy and preconditioner against the oracle."""
    _say(f"case one-sided pattern {spec}")
    s = nfgen.tsi2d(nel=16, seed=2, nrhs=2)
    for i in range(2):
        s.blocks[i][i] = nfgen.one_sided_pattern(s.blocks[i][i], 10 + i, frac=0.3)
    opts = dict(coarse_max=40, **TSI_OPTS)
    o = oracle.Oracle(s.fields, s.blocks, spec, **opts)
    g = _gpu(s, spec, **opts)
    _compare_hierarchies(g, o)
    r = np.random.default_rng(12).standard_normal((2, s.n))
    zo = o.precond_apply(r)
    zg = g.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    for k in range(2):
        assert np.linalg.norm(zg[k] - zo[k]) <= 1e-10 * np.linalg.norm(zo[k]), k


# ------------------------------- coupling-strength sweep (Sec. 7.1, TSI)
# the preconditioners of the sweep, each against the oracle at a weak, a
# medium and a strong coupling (where some of them stop converging)
ALPHA_SPECS = [("BGS(AMG)", dict(sweeps=2, order="bwd")), ("BGS[order=sym](AMG)", dict(sweeps=2)),
               ("AMG(BGS)", dict(sweeps=2, order="bwd")), ("SIMPLE(AMG;AMG)", {})]


@pytest.mark.parametrize("alpha", [1e-2, 30.0, 300.0])
@pytest.mark.parametrize("spec,opts", ALPHA_SPECS)
def test_alpha_sweep_parity(dev, spec, opts, alpha):
    _say(f"case alpha sweep {spec} alpha={alpha}")
    s = nfgen.tsi2d_alpha(alpha, nel=32, nrhs=1)
    o = oracle.Oracle(s.fields, s.blocks, spec, **opts)
    g = _gpu(s, spec, **opts)
    r = np.random.default_rng(13).standard_normal(s.n)
    zo = o.precond_apply(r)
    zg = g.precond_apply(torch.tensor(r, device=dev)).cpu().numpy()
    assert np.linalg.norm(zg - zo) <= 1e-10 * np.linalg.norm(zo)
    A = s.assembled()
    x, st = g.gmres_solve(torch.tensor(s.rhs[0], device=dev), rtol=1e-8, maxit=300)
    x = x.cpu().numpy()
    xo, so = o.gmres(s.rhs[0], rtol=1e-8, maxit=300)
    _say(f"  gpu {st[0]['status']}/{st[0]['iters']} oracle {so['status']}/{so['iters']}")
    if so["status"] == 0 and so["iters"] < 290:
        res = np.linalg.norm(s.rhs[0] - A @ x) / np.linalg.norm(s.rhs[0])
        assert st[0]["status"] == 0 and res < 1e-8
        assert np.linalg.norm(x - xo) <= 1e-6 * np.linalg.norm(xo)
        assert abs(st[0]["iters"] - so["iters"]) <= 2
    else:
        # both stop at the iteration limit (or both converge at its very end)
        assert so["iters"] >= 290 and st[0]["iters"] >= 288


def test_rebuild_after_value_update(dev):
    _say("case rebuild after update_values")
    s = nfgen.tsi2d(nel=20, seed=3)
    g = _gpu(s, "BGS(AMG)", **TSI_OPTS)
    s2 = nfgen.tsi2d(nel=20, seed=3, E=2.0, alpha=3e-2)
    for i in range(2):
        for j in range(2):
            g.update_values(i, j, torch.tensor(s2.blocks[i][j].data, device=dev))
    g.rebuild()
    o = oracle.Oracle(s2.fields, s2.blocks, "BGS(AMG)", **TSI_OPTS)
    _compare_hierarchies(g, o)
    x, st = g.gmres_solve(torch.tensor(s2.rhs[0], device=dev))
    xo, _ = o.gmres(s2.rhs[0])
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-6 * np.linalg.norm(xo)


# ------------------------------------------------------------ batched columns
@pytest.mark.parametrize("spec,make", [
    ("BGS(AMG)", lambda: nfgen.tsi2d(nel=24, seed=8, nrhs=7)),
    (FSI_SPEC, lambda: nfgen.fsi3d(n=8, layers=2, seed=0, nrhs=5))])
def test_batched_columns_equal_solo_bitwise(dev, spec, make):
    """Each right-hand side gives the same bits alone and inside a batch."""
    _say(f"case batched vs solo {spec}")
    s = make()
    opts = dict(TSI_OPTS) if "BGS(AMG)" == spec else dict(FSI_OPTS)
    g = _gpu(s, spec, **opts)
    B = torch.tensor(s.rhs, device=dev)
    xb, stb = g.gmres_solve(B, rtol=1e-8)
    zb = g.precond_apply(B)
    A = s.assembled()
    for k in range(s.rhs.shape[0]):
        xs, sts = g.gmres_solve(B[k].contiguous(), rtol=1e-8)
        zs = g.precond_apply(B[k].contiguous())
        assert torch.equal(xs, xb[k]), k
        assert torch.equal(zs, zb[k]), k
        assert sts[0]["iters"] == stb[k]["iters"]
        xk = xb[k].cpu().numpy()
        assert stb[k]["status"] == 0
        assert np.linalg.norm(s.rhs[k] - A @ xk) / np.linalg.norm(s.rhs[k]) < 1e-8


def test_batched_precision_form(dev):
    _say("case batched precision form fsi3d")
    s = nfgen.fsi3d(n=10, layers=2, seed=0, nrhs=3)
    o = oracle.Oracle(s.fields, s.blocks, FSI_SPEC, **FSI_OPTS)
    g = _gpu(s, FSI_SPEC, hier_fp32=1, **FSI_OPTS)
    A = s.assembled()
    x, st = g.gmres_solve(torch.tensor(s.rhs, device=dev), flexible=1, rtol=1e-8)
    x = x.cpu().numpy()
    for k in range(3):
        xo, so = o.gmres(s.rhs[k], rtol=1e-8)
        res = np.linalg.norm(s.rhs[k] - A @ x[k]) / np.linalg.norm(s.rhs[k])
        err = np.linalg.norm(x[k] - xo) / np.linalg.norm(xo)
        _say(f"  rhs {k}: iters {st[k]['iters']} (oracle fp64 {so['iters']}) relres {res:.2e} err {err:.2e}")
        assert st[k]["status"] == 0 and res < 1e-8 and err < 1e-6
