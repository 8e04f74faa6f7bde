"""Seeded N x N block systems that stand in for the paper's coupled problems.

Each builder returns a :class:`BlockSystem`: per-field sizes, block sizes and
near-nullspace vectors, the N x N grid of CSR blocks (``None`` = zero block)
and seeded right-hand sides.  The block shapes follow the paper's coupled
systems: the 2x2 thermo-structure Jacobian (Section 6, TSI monolithic system),
the 3x3 solid / grid / fluid FSI system (Section 6, FSI block system) and the
lung's FSI-plus-constraint saddle point (Section 6, lung block system).  The
physics is synthetic; only the structure and scales are meant to match.
"""
from dataclasses import dataclass, field as dfield
import numpy as np
import scipy.sparse as sp

from . import fem


@dataclass
class Field:
    name: str
    ndof: int
    block_size: int
    nullspace: np.ndarray          # (nns, ndof), row c = near-nullspace vector c

    @property
    def nns(self):
        return self.nullspace.shape[0]


@dataclass
class BlockSystem:
    fields: list
    blocks: list                   # blocks[i][j]: scipy CSR (float64) or None
    rhs: np.ndarray                # (nrhs, n): row c = right-hand side c
    meta: dict = dfield(default_factory=dict)

    @property
    def nfields(self):
        return len(self.fields)

    @property
    def n(self):
        return sum(f.ndof for f in self.fields)

    def offsets(self):
        o = [0]
        for f in self.fields:
            o.append(o[-1] + f.ndof)
        return o

    def nnz(self):
        return sum(b.nnz for row in self.blocks for b in row if b is not None)

    def assembled(self):
        """The whole matrix as one CSR (for dense/LU comparisons in tests)."""
        rows = []
        for i, fi in enumerate(self.fields):
            rows.append([self.blocks[i][j] if self.blocks[i][j] is not None
                         else sp.csr_matrix((fi.ndof, fj.ndof)) for j, fj in enumerate(self.fields)])
        M = sp.bmat(rows, format="csr")
        M.sort_indices()
        return M


def permute_fields(sys_, order):
    """The same system with its fields (and block rows / columns, right-hand
    side slices) taken in the given order."""
    o = sys_.offsets()
    rhs = np.concatenate([sys_.rhs[:, o[i]:o[i + 1]] for i in order], axis=1)
    blocks = [[sys_.blocks[i][j] for j in order] for i in order]
    return BlockSystem([sys_.fields[i] for i in order], blocks, rhs, meta=dict(sys_.meta, field_order=list(order)))


def one_sided_pattern(A, seed, frac=0.3):
    """A copy of A with a seeded share `frac` of its strictly upper entries
    removed: a nonsymmetric pattern in which row u couples to v while row v
    no longer couples to u."""
    A = sp.coo_matrix(A)
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x051DE]))
    drop = (A.col > A.row) & (rng.random(A.nnz) < frac)
    B = sp.csr_matrix((A.data[~drop], (A.row[~drop], A.col[~drop])), shape=A.shape)
    B.sort_indices()
    return B


def uniform_rhs(n, nrhs, seed):
    """iid uniform[-1, 1] right-hand sides, (nrhs, n)."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x5EED]))
    return rng.uniform(-1.0, 1.0, size=(nrhs, n))


def rigid_modes_2d(xy, center):
    """Planar rigid-body modes (2 translations + rotation), interleaved dofs."""
    n = xy.shape[0]
    B = np.zeros((3, 2 * n))
    B[0, 0::2] = 1.0
    B[1, 1::2] = 1.0
    B[2, 0::2] = -(xy[:, 1] - center[1])
    B[2, 1::2] = xy[:, 0] - center[0]
    return B


def rigid_modes_3d(xyz, center):
    """3 translations + 3 infinitesimal rotations, interleaved dofs."""
    n = xyz.shape[0]
    d = xyz - np.asarray(center)[None, :]
    B = np.zeros((6, 3 * n))
    for c in range(3):
        B[c, c::3] = 1.0
    # rotation about z: (-y, x, 0); about x: (0, -z, y); about y: (z, 0, -x)
    B[3, 0::3] = -d[:, 1]
    B[3, 1::3] = d[:, 0]
    B[4, 1::3] = -d[:, 2]
    B[4, 2::3] = d[:, 1]
    B[5, 0::3] = d[:, 2]
    B[5, 2::3] = -d[:, 0]
    return B


# --------------------------------------------------------------------------
# 2-field thermo-structure-like system (the TSI 2x2 block Jacobian)
# --------------------------------------------------------------------------
def tsi2d(nel=32, E=1.0, nu=0.3, kappa=1.0, dt=0.1, alpha=1e-2, cba=1e-3,
          cba_sign=+1.0, seed=0, nrhs=1, clamp=True, heat_mass=True,
          coupling=True):
    """Plane-strain elasticity (field A, 2 dof/node) + transient heat (field B).

    Unit square, nel x nel bilinear elements.  A is clamped at x = 0 (those
    dofs are removed).  B = M/dt + kappa*K on all nodes.
    C_AB = alpha * int B^T m N  with m = (1, 1, 0) (thermal stress),
    C_BA = cba_sign * cba * int N div(N_u)  (mass-weighted divergence).
    clamp=False / heat_mass=False give the singular Neumann operators whose
    kernels are the rigid-body / constant modes (used to test prolongators).
    """
    h = 1.0 / nel
    nn1 = nel + 1
    nnodes = nn1 * nn1
    ii, jj = np.meshgrid(np.arange(nn1), np.arange(nn1), indexing="xy")
    xy = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1)
    conn = fem.grid_conn_2d(nel, nel)
    g = fem.q1_2d(h, h)

    free_node = np.ones(nnodes, bool)
    if clamp:
        free_node[ii.ravel() == 0] = False
    free_dof = np.repeat(free_node, 2)
    umap = fem.renumber(free_dof)
    nA = int(free_dof.sum())
    nB = nnodes

    edofs = fem.element_dofs(conn, 2)
    Ke = fem.ke_elastic(g, E, nu)
    AAA = fem.assemble(edofs, edofs, Ke, nA, nA, umap, umap)

    Kt = fem.ke_laplace(g, kappa)
    Mt = fem.ke_mass(g)
    Bt = kappa * Kt + (Mt / dt if heat_mass else 0.0 * Mt)
    ABB = fem.assemble(conn, conn, Bt, nB, nB)

    blocks = [[AAA, None], [None, ABB]]
    if coupling:
        G = fem.ke_grad_shape(g)                        # (8, 4)
        CAB = fem.assemble(edofs, conn, alpha * G, nA, nB, umap, None)
        CBA = fem.assemble(conn, edofs, cba_sign * cba * G.T, nB, nA, None, umap)
        blocks = [[AAA, CAB], [CBA, ABB]]

    nsA = rigid_modes_2d(xy[free_node], (0.5, 0.5))
    nsB = np.ones((1, nB))
    fields = [Field("structure", nA, 2, nsA), Field("thermo", nB, 1, nsB)]
    sys_ = BlockSystem(fields, blocks, uniform_rhs(nA + nB, nrhs, seed),
                       meta=dict(kind="tsi2d", nel=nel, seed=seed))
    return sys_


def tsi2d_alpha(alpha, nel=32, seed=0, nrhs=1):
    """The TSI-like system at coupling strength alpha: as in the paper's
    thermo-mechanical system both off-diagonal blocks grow with the thermal
    expansion coefficient, here C_AB = alpha int B^T m N and
    C_BA = -0.1 alpha int N div(N_u) (opposite signs, as thermal stress and
    thermoelastic heating have, so that the coupled operator stays
    well-posed as alpha grows and only the block splittings suffer).
    alpha = 1e-2 gives the default coupling magnitudes of tsi2d."""
    return tsi2d(nel=nel, alpha=alpha, cba=0.1 * alpha, cba_sign=-1.0, seed=seed, nrhs=nrhs)


ALPHA_SWEEP = (1e-2, 1e-1, 1.0, 10.0, 30.0, 100.0, 300.0, 1000.0)


# --------------------------------------------------------------------------
# 3-field FSI-like system (solid S, grid motion G, fluid F)
# --------------------------------------------------------------------------
def _advection_field(centers, seed, kmax=2):
    """a = curl(psi), psi_c = sum_k alpha_{c,k} sin(pi k.x) over integer wave
    vectors with 0 < |k| <= kmax, scaled so that max |a| = 1 over the points."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0xADF]))
    ks = [np.array(k) for k in np.ndindex(kmax + 1, kmax + 1, kmax + 1)
          if 0 < np.linalg.norm(k) <= kmax]
    a = np.zeros_like(centers)
    for k in ks:
        alpha = rng.standard_normal(3)
        phase = np.pi * centers @ k
        c = np.cos(phase)
        # grad psi_c = alpha_c pi k cos(pi k.x);  curl: (d_y psi_z - d_z psi_y, ...)
        g = np.pi * c[:, None] * k[None, :]
        a[:, 0] += alpha[2] * g[:, 1] - alpha[1] * g[:, 2]
        a[:, 1] += alpha[0] * g[:, 2] - alpha[2] * g[:, 0]
        a[:, 2] += alpha[1] * g[:, 0] - alpha[0] * g[:, 1]
    return a / np.max(np.linalg.norm(a, axis=1))


def fsi3d(n=40, layers=8, nu=1e-2, E=1e3, nu_s=0.3, dt=1.0, seed=0, nrhs=1):
    """Fluid (PSPG-stabilised Q1-Q1 Oseen, 4 dof/node) on an n^3 hex box,
    ALE grid motion (vector Laplacian) on the same mesh, and a Q1 elastic slab
    of n x n x layers elements on the fluid's top face.

    Fluid: no-slip on the five faces other than the top; those velocity dofs
    stay as identity rows (uniform 4 dofs per node).  ALE: zero on the same
    five faces; its interior nodes are the G unknowns.  Structure: lateral
    faces clamped; its bottom (interface) nodes match the fluid's top-face
    nodes.  The interface displacements of S and G are condensed onto the
    fluid interface velocities, d = dt * u (the solid-interface rows are
    added to the fluid interface momentum rows), which gives the block
    pattern [SS 0 SF; 0 GG GF; FS 0 FF].  Field order (S, G, F).
    """
    h = 1.0 / n
    # ---------------- fluid grid: 4 dofs per node (u, v, w, p)
    fdims = (n + 1, n + 1, n + 1)
    fijk = fem.grid_nodes(fdims)
    nfn = fijk.shape[0]
    wall = (fijk[:, 0] == 0) | (fijk[:, 0] == n) | (fijk[:, 1] == 0) | (fijk[:, 1] == n) | (fijk[:, 2] == 0)
    top_int = (fijk[:, 2] == n) & ~wall
    conn = fem.grid_conn_3d(n, n, n)
    centers = (fijk[conn[:, 0]] + 0.5) * h
    a = _advection_field(centers, seed)
    amag = np.linalg.norm(a, axis=1)
    tau = ((2 * amag / h) ** 2 + (4 * nu / h ** 2) ** 2) ** -0.5
    L, Cm, G, D, _ = fem.gauss_tensors_3d(h)

    def fluid_pair(ia, ib):
        blk = np.zeros((conn.shape[0], 4, 4))
        conv = a @ Cm[:, ia, ib]                                  # sum_d a_d int N_a dN_b/dx_d
        for c in range(3):
            blk[:, c, c] = nu * L[ia, ib] + conv
            blk[:, c, 3] = -G[c, ia, ib]                          # -int dN_a/dx_c N_b
            blk[:, 3, c] = G[c, ib, ia] + tau * (a @ D[c, :, ia, ib])   # div + PSPG convection
        blk[:, 3, 3] = tau * L[ia, ib]                            # PSPG pressure Laplacian
        return blk

    stF, _ = fem.stencil_assemble((n, n, n), 4, fluid_pair)
    fdir = np.zeros(nfn * 4, bool)
    for c in range(3):
        fdir[np.nonzero(wall)[0] * 4 + c] = True
    nF = nfn * 4
    ident = np.arange(nF)
    fpairs = np.ones((4, 4), bool)
    fpairs[:3, :3] = np.eye(3, dtype=bool)
    AFF = fem.stencil_to_csr(stF, fdims, ident, ident, nF, nF, fpairs, dirichlet=fdir)
    del stF

    # fluid interface velocity dof of each top-face node
    def fluid_vel_dof(node, c):
        return node * 4 + c

    # ---------------- ALE on the fluid grid: 3 dofs per node
    Lap = L.copy()
    stG, _ = fem.stencil_assemble((n, n, n), 3, lambda ia, ib: np.broadcast_to(
        np.eye(3) * Lap[ia, ib], (conn.shape[0], 3, 3)))
    interior = (fijk[:, 0] > 0) & (fijk[:, 0] < n) & (fijk[:, 1] > 0) & (fijk[:, 1] < n) & \
               (fijk[:, 2] > 0) & (fijk[:, 2] < n)
    g_int_dof = np.repeat(interior, 3)
    gmap = fem.renumber(g_int_dof)
    nG = int(g_int_dof.sum())
    g_if = np.full(nfn * 3, -1, np.int64)            # ALE interface dof -> fluid velocity dof
    ifn = np.nonzero(top_int)[0]
    for c in range(3):
        g_if[ifn * 3 + c] = fluid_vel_dof(ifn, c)
    gpairs = np.eye(3, dtype=bool)
    AGG = fem.stencil_to_csr(stG, fdims, gmap, gmap, nG, nG, gpairs)
    AGF = fem.stencil_to_csr(stG, fdims, gmap, g_if, nG, nF, gpairs) * dt
    del stG

    # ---------------- structure slab: nodes (i, j, k), k = 0 on the interface
    sdims = (n + 1, n + 1, layers + 1)
    sijk = fem.grid_nodes(sdims)
    nsn = sijk.shape[0]
    clamped = (sijk[:, 0] == 0) | (sijk[:, 0] == n) | (sijk[:, 1] == 0) | (sijk[:, 1] == n)
    s_free = ~clamped & (sijk[:, 2] > 0)
    s_if = ~clamped & (sijk[:, 2] == 0)
    Ke = fem.ke_elastic(fem.q1_3d(h, h, h), E, nu_s).reshape(8, 3, 8, 3)
    sconn = fem.grid_conn_3d(n, n, layers)
    stS, _ = fem.stencil_assemble((n, n, layers), 3, lambda ia, ib: np.broadcast_to(
        Ke[ia, :, ib, :], (sconn.shape[0], 3, 3)))
    smap = fem.renumber(np.repeat(s_free, 3))
    nS = int(np.repeat(s_free, 3).sum())
    # structure interface node (i, j, 0) <-> fluid node (i, j, n)
    s_to_f = np.full(nsn * 3, -1, np.int64)
    sn_if = np.nonzero(s_if)[0]
    fnode = (n * (n + 1) + sijk[sn_if, 1]) * (n + 1) + sijk[sn_if, 0]
    for c in range(3):
        s_to_f[sn_if * 3 + c] = fluid_vel_dof(fnode, c)
    ASS = fem.stencil_to_csr(stS, sdims, smap, smap, nS, nS)
    ASF = fem.stencil_to_csr(stS, sdims, smap, s_to_f, nS, nF) * dt
    AFS = fem.stencil_to_csr(stS, sdims, s_to_f, smap, nF, nS)
    AFF_s = fem.stencil_to_csr(stS, sdims, s_to_f, s_to_f, nF, nF) * dt
    del stS
    AFF = (AFF + AFF_s).tocsr()
    AFF.sort_indices()

    xyz_s = sijk[s_free] * h + np.array([0.0, 0.0, 1.0])
    nsS = rigid_modes_3d(xyz_s, xyz_s.mean(axis=0))
    nsG = np.zeros((3, nG))
    for c in range(3):
        nsG[c, c::3] = 1.0
    nsF = np.zeros((4, nF))
    for c in range(4):
        nsF[c, c::4] = 1.0
    nsF[:, fdir] = 0.0
    fields = [Field("solid", nS, 3, nsS), Field("grid", nG, 3, nsG), Field("fluid", nF, 4, nsF)]
    blocks = [[ASS, None, ASF], [None, AGG, AGF], [AFS, None, AFF]]
    for row in blocks:
        for B in row:
            if B is not None:
                B.sort_indices()
    return BlockSystem(fields, blocks, uniform_rhs(nS + nG + nF, nrhs, seed),
                       meta=dict(kind="fsi3d", n=n, layers=layers, seed=seed,
                                 split=[0, 0, 1]))


# --------------------------------------------------------------------------
# Serving trace: TSI-like systems of several grid sizes with Poisson arrivals
# --------------------------------------------------------------------------
SERVE_GRIDS = (16, 24, 32, 48, 64, 96, 128)


def request_trace(n_requests=512, rate=100.0, grids=SERVE_GRIDS, max_rhs=8, seed=0):
    """Requests with Poisson arrivals (rate per second), a grid size drawn
    uniformly from `grids` and 1..max_rhs right-hand sides each.  Every
    request is a 2-field TSI-like system (tsi2d) of its grid size; its
    right-hand sides come from its own seed (see request_rhs)."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x7EACE]))
    gaps = rng.exponential(1.0 / rate, n_requests)
    arrival = np.concatenate([[0.0], np.cumsum(gaps[1:])])
    grid = rng.choice(np.asarray(grids), n_requests)
    nrhs = rng.integers(1, max_rhs + 1, n_requests)
    rseed = rng.integers(0, 2**31 - 1, n_requests)
    return [dict(id=i, arrival_s=float(arrival[i]), grid=int(grid[i]), nrhs=int(nrhs[i]),
                 rhs_seed=int(rseed[i])) for i in range(n_requests)]


def request_rhs(req, n):
    """The request's right-hand sides, (nrhs, n)."""
    return uniform_rhs(n, req["nrhs"], req["rhs_seed"])


# --------------------------------------------------------------------------
# Lung-like system: tissue (T), airway tree (W), volume constraints (L)
# --------------------------------------------------------------------------
def _acinus_constraint_rows(n, nacini, m, seed, free_map):
    """B_k u = volume change of acinus k (an m^3 element sub-block of the n^3
    box), written as the surface integral of u.n over the sub-block's
    faces: for a face node, +-h^2 times its trapezoid weight on that face
    (1 inside the face, 1/2 on a face edge, 1/4 at a face corner) in the
    component normal to the face.  Origins are drawn without replacement."""
    h = 1.0 / n
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0xAC1]))
    span = n - m + 1
    flat = rng.choice(span ** 3, size=nacini, replace=False)
    org = np.stack([flat % span, (flat // span) % span, flat // (span * span)], axis=1)
    ln = np.arange(m + 1)
    wts = np.where((ln == 0) | (ln == m), 0.5, 1.0)
    rows, cols, vals = [], [], []
    n1 = n + 1
    for k, (ox, oy, oz) in enumerate(org):
        entries = {}
        for c in range(3):                       # faces normal to axis c
            a1, a2 = [d for d in range(3) if d != c]
            for side, sign in ((0, -1.0), (m, 1.0)):
                g1, g2 = np.meshgrid(ln, ln, indexing="ij")
                idx = np.zeros((3,) + g1.shape, int)
                idx[c] = side
                idx[a1] = g1
                idx[a2] = g2
                gi = idx[0] + ox
                gj = idx[1] + oy
                gk = idx[2] + oz
                node = (gk * n1 + gj) * n1 + gi
                w = sign * h * h * wts[g1] * wts[g2]
                for nd, ww in zip(node.ravel(), w.ravel()):
                    dof = free_map[nd * 3 + c]
                    if dof >= 0:
                        entries[dof] = entries.get(dof, 0.0) + ww
        ks = sorted(entries)
        rows += [k] * len(ks)
        cols += ks
        vals += [entries[q] for q in ks]
    return rows, cols, vals


def lung3d(n=64, depth=12, acinus=8, E=1.0, nu=0.45, dt=1.0, seed=0, nrhs=1, rt_scale=None):
    """Tissue: Q1 linear elasticity (the Neo-Hookean model linearised at the
    reference state) on an n^3 box, clamped at z = 0, K u - B^T lambda = f.

    Airway: a binary tree of the given depth (2^(depth+1) - 1 segments in heap
    order, root 0, children 2s+1 and 2s+2), 2 dofs per segment: the pressure
    p_s at its distal node and its flow q_s (towards the acini).  Segment
    resistances R_s are log-uniform in [1e-2, 1]; the pressure upstream of the
    root (the mouth) is 0.  Terminal segment k feeds acinus k through an
    acinar resistance Rt_k = rt_scale * (log-uniform in [1e-2, 1]); the default
    rt_scale = 2^depth makes the 2^depth acini in parallel as resistive as one
    segment.  The multiplier lambda_k is the pressure in acinus k.

    The airway block is the Hessian of the convex quadratic
        Phi(p, q) = 1/2 sum_s R_s (q_s - dp_s / R_s)^2 + 1/2 p^T L p,
    dp_s = pressure drop along the segment (or along segment + acinus), L the
    weighted tree Laplacian grounded at the mouth and (through Rt_k) at the
    acini, so it is symmetric positive definite.  Its stationarity conditions
    are exactly the physics: Poiseuille on every segment,
        R_s q_s - (p_parent - p_s) = 0                  (internal flow rows)
        (R_s + Rt_k) q_s - (p_parent - lambda_k) = 0    (terminal flow rows)
    and mass conservation at every node, which the pressure rows state as
        2 (L p)_s + q_s - sum_c q_c = 0                 (internal)
        2 (L p)_s = 0                                   (terminal)
    (on a solution q_s - sum_c q_c = -(L p)_s, so both read (L p)_s = 0).

    Constraints: one per acinus, B_k u - dt q_k = 0 (volume change of the
    acinus equals its inflow over the step), B_k the analytic surface form of
    the acinus' volume change.  The multiplier block is zero (a saddle point).
    """
    h = 1.0 / n
    nterm = 2 ** depth
    nseg = 2 ** (depth + 1) - 1
    if rt_scale is None:
        rt_scale = float(nterm)
    dims = (n + 1, n + 1, n + 1)
    ijk = fem.grid_nodes(dims)
    free = ijk[:, 2] > 0
    free_dof = np.repeat(free, 3)
    tmap = fem.renumber(free_dof)
    nT = int(free_dof.sum())
    Ke = fem.ke_elastic(fem.q1_3d(h, h, h), E, nu).reshape(8, 3, 8, 3)
    conn = fem.grid_conn_3d(n, n, n)
    st, _ = fem.stencil_assemble((n, n, n), 3, lambda ia, ib: np.broadcast_to(Ke[ia, :, ib, :], (conn.shape[0], 3, 3)))
    ATT = fem.stencil_to_csr(st, dims, tmap, tmap, nT, nT)
    del st
    # airway tree
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0xA1B]))
    R = np.exp(rng.uniform(np.log(1e-2), np.log(1.0), nseg))
    Rt = rt_scale * np.exp(rng.uniform(np.log(1e-2), np.log(1.0), nterm))
    nW = 2 * nseg
    first_term = nseg - nterm
    g = 1.0 / R
    wr, wc, wv = [], [], []
    lr, lc, lv = [], [], []          # airway -> multiplier coupling
    for sgm in range(nseg):
        p, q = 2 * sgm, 2 * sgm + 1
        par = (sgm - 1) // 2 if sgm > 0 else -1
        # pressure rows: twice the weighted tree Laplacian plus the flow
        # balance q_s - sum_c q_c (internal nodes only)
        wr.append(p); wc.append(p); wv.append(2.0 * g[sgm])
        if par >= 0:
            # Laplacian couplings and the segment's share of the parent's diagonal
            wr += [p, 2 * par, 2 * par]
            wc += [2 * par, p, 2 * par]
            wv += [-2.0 * g[sgm], -2.0 * g[sgm], 2.0 * g[sgm]]
        if sgm < first_term:
            wr.append(p); wc.append(q); wv.append(1.0)
            for c in (2 * sgm + 1, 2 * sgm + 2):
                wr.append(p); wc.append(2 * c + 1); wv.append(-1.0)
            # flow row: Poiseuille, R_s q_s - (p_parent - p_s) = 0
            wr += [q, q]; wc += [q, p]; wv += [R[sgm], 1.0]
            if par >= 0:
                wr.append(q); wc.append(2 * par); wv.append(-1.0)
        else:
            k = sgm - first_term
            wr.append(p); wc.append(p); wv.append(2.0 / Rt[k])
            lr.append(p); lc.append(k); lv.append(-2.0 / Rt[k])
            # flow row: segment and acinus in series, (R_s + Rt_k) q_s - p_parent + lambda_k = 0
            wr.append(q); wc.append(q); wv.append(R[sgm] + Rt[k])
            if par >= 0:
                wr.append(q); wc.append(2 * par); wv.append(-1.0)
            lr.append(q); lc.append(k); lv.append(1.0)
    AWW = sp.csr_matrix((wv, (wr, wc)), shape=(nW, nW))
    AWW.sum_duplicates()
    AWW.sort_indices()
    AWL = sp.csr_matrix((lv, (lr, lc)), shape=(nW, nterm))
    AWL.sort_indices()
    # constraints
    br, bc, bv = _acinus_constraint_rows(n, nterm, acinus, seed, tmap)
    B = sp.csr_matrix((bv, (br, bc)), shape=(nterm, nT))
    B.sort_indices()
    ALT = B
    ATL = sp.csr_matrix(-B.T)
    ATL.sort_indices()
    ALW = sp.csr_matrix((-dt * np.ones(nterm), (np.arange(nterm), 2 * (first_term + np.arange(nterm)) + 1)),
                        shape=(nterm, nW))
    ALW.sort_indices()
    xyz = ijk[free] * h
    nsT = rigid_modes_3d(xyz, xyz.mean(axis=0))
    nsW = np.zeros((2, nW))
    nsW[0, 0::2] = 1.0
    nsW[1, 1::2] = 1.0
    nsL = np.ones((1, nterm))
    fields = [Field("tissue", nT, 3, nsT), Field("airway", nW, 2, nsW), Field("multiplier", nterm, 1, nsL)]
    blocks = [[ATT, None, ATL], [None, AWW, AWL], [ALT, ALW, None]]
    return BlockSystem(fields, blocks, uniform_rhs(nT + nW + nterm, nrhs, seed),
                       meta=dict(kind="lung3d", n=n, depth=depth, seed=seed, split=[0, 0, 1]))
