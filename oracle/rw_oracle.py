"""CPU oracle for the random-walker Dirichlet solve — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The GPU library never calls it and
shares no code with it.

What it computes (random-walker segmentation as cited in the paper's operator
list, Sec. III-A, and the hierarchical variant benchmarked in Sec. IV-B,
Table III):

* The graph is the 6-connected voxel grid.  Edge (i, j) carries the Gaussian
  weight ``w_ij = exp(-beta (g_i - g_j)^2) (+ w_eps)`` of the normalised
  intensities ``g``; edges never leave the volume (natural boundary).
* ``L = D - W`` is the graph Laplacian.  With voxels split into seeded ``M``
  and unseeded ``U``, label ``s`` has Dirichlet data ``m^s_j = [label_j = s]``
  on ``M`` and its probability map solves ``L_U x_U = -B^T m^s``
  (combinatorial Dirichlet problem).
* The exact answer of that system is the plain definition; the method reaches
  it approximately, by Jacobi-preconditioned conjugate gradients stopped at
  ``||r|| <= tol ||b||``.  This module provides both: a direct sparse / dense
  solve ("O-exact") and the Jacobi-PCG written step by step ("O-same").

Everything is float64.  The formulation is the explicitly assembled sparse
matrix (COO -> CSR, index sets for U and M), deliberately unlike the GPU's
matrix-free stencil.

Pins (tests/test_oracle_*.py): dense direct solve, closed-form linear ramp,
1D resistor divider, maximum principle, sum-to-one, axis-permutation
equivariance, beta = 0 image independence, Monte-Carlo walks, domain
decomposition identity, complex-step gradients.  The hierarchical pipeline's
agreement with the true fine-level solution is "parity unpinned": only its
steps are pinned (see hierarchical_rw).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# status codes shared in meaning (not in code) with the C ABI
OK = 0
NOT_CONVERGED = 1
ERR_INVALID_ARG = -1
ERR_NO_SEEDS = -2
ERR_SINGULAR = -3
ERR_BREAKDOWN = -4
ERR_NONFINITE = -5


class OracleError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"oracle status {status}: {msg}")
        self.status = status


# --------------------------------------------------------------------------
# normalisation and weights
# --------------------------------------------------------------------------

def normalize(vol, lo, hi):
    """g = (v - lo) / (hi - lo) in float64; a constant image (hi <= lo) gives g = 0."""
    v = np.asarray(vol, dtype=np.float64)
    if not hi > lo:
        return np.zeros_like(v)
    return (v - lo) / (hi - lo)


def case_g(case):
    """Normalised intensities of a synthetic case (min-max for float, /65535 for u16)."""
    lo, hi = case.norm_range()
    return normalize(case.vol, lo, hi)


def grid_edges(shape):
    """Every undirected grid edge once, as flat index pairs (i, j = i + e_axis),
    for a 3-D grid [nz][ny][nx] (6-connected) or a 4-D time series
    [nt][nz][ny][nx] (8-connected: the two neighbours along each axis).

    Returns (i, j, axis) with axis 0 = x (the fastest array axis), 1 = y,
    2 = z and, in 4-D, 3 = t.
    """
    shape = tuple(int(n) for n in shape)
    idx = np.arange(int(np.prod(shape)), dtype=np.int64).reshape(shape)
    nd = len(shape)
    ii, jj, aa = [], [], []
    for axis in range(nd):
        ax = nd - 1 - axis  # array axis of grid axis `axis`
        lo = [slice(None)] * nd
        hi = [slice(None)] * nd
        lo[ax] = slice(None, -1)
        hi[ax] = slice(1, None)
        a, b = idx[tuple(lo)], idx[tuple(hi)]
        ii.append(a.ravel())
        jj.append(b.ravel())
        aa.append(np.full(a.size, axis, dtype=np.int8))
    return np.concatenate(ii), np.concatenate(jj), np.concatenate(aa)


def edge_weights(g, beta, w_eps=0.0, edges=None, dtype=np.float64):
    """Gaussian weight of every edge: exp(-beta (g_i - g_j)^2) + w_eps."""
    if edges is None:
        edges = grid_edges(g.shape)
    i, j, _ = edges
    gf = np.asarray(g).ravel()
    diff = gf[i].astype(dtype) - gf[j].astype(dtype)
    return np.exp(-dtype(beta) * diff * diff) + dtype(w_eps)


def weights_grid(g, beta, w_eps=0.0):
    """Weights laid out as w[3][nz][ny][nx]: w[a][v] belongs to edge (v, v + e_a),
    a = 0 (x), 1 (y), 2 (z); the last plane along each axis is 0 (no edge)."""
    g = np.asarray(g, dtype=np.float64)
    w = np.zeros((3,) + g.shape)
    w[0][:, :, :-1] = np.exp(-beta * (g[:, :, 1:] - g[:, :, :-1]) ** 2) + w_eps
    w[1][:, :-1, :] = np.exp(-beta * (g[:, 1:, :] - g[:, :-1, :]) ** 2) + w_eps
    w[2][:-1, :, :] = np.exp(-beta * (g[1:, :, :] - g[:-1, :, :]) ** 2) + w_eps
    return w


def laplacian(shape, w, edges=None):
    """Assembled graph Laplacian L = D - W (CSR) from per-edge weights."""
    if edges is None:
        edges = grid_edges(shape)
    i, j, _ = edges
    n = int(np.prod(shape))
    rows = np.concatenate([i, j, i, j])
    cols = np.concatenate([j, i, i, j])
    vals = np.concatenate([-w, -w, w, w])
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()


# --------------------------------------------------------------------------
# the Dirichlet system
# --------------------------------------------------------------------------

class DirichletSystem:
    """L_U, B = L_UM, index sets and Dirichlet vectors of one volume."""

    def __init__(self, g, labels, beta, w_eps=0.0, K=None):
        self.shape = g.shape
        self.labels = np.asarray(labels).ravel()
        self.K = int(K if K is not None else self.labels.max())
        self.edges = grid_edges(g.shape)
        self.w = edge_weights(g, beta, w_eps, self.edges)
        self.L = laplacian(g.shape, self.w, self.edges)
        self.M = np.flatnonzero(self.labels > 0)
        self.U = np.flatnonzero(self.labels == 0)
        if self.M.size == 0:
            raise OracleError(ERR_NO_SEEDS, "no seeds")
        self.LU = self.L[self.U][:, self.U].tocsr()
        self.B = self.L[self.U][:, self.M].tocsr()
        self.diag = self.LU.diagonal()

    def m(self, s):
        """Dirichlet data of label s on M: the indicator [label = s]."""
        return (self.labels[self.M] == s).astype(np.float64)

    def rhs(self, s):
        """b = -B m^s."""
        return -(self.B @ self.m(s))

    def full(self, s, xU):
        """Full grid: seeds exact, unknowns from xU."""
        x = np.empty(self.labels.size)
        x[self.M] = self.m(s)
        x[self.U] = xU
        return x.reshape(self.shape)


def pcg_jacobi(A, b, dinv, x0, tol, max_iter):
    """Jacobi-preconditioned CG (Hestenes-Stiefel) in float64.

    Steps: r = b - A x0, z = D^-1 r, p = z, rho = r.z; then per iteration
    q = A p, sigma = p.q (breakdown if sigma <= 0 or not finite),
    alpha = rho / sigma, x += alpha p, r -= alpha q, stop when
    ||r|| <= tol ||b||, else z = D^-1 r, rho' = r.z, p = z + (rho'/rho) p.

    Returns (x, iterations, status).  ``||b|| = 0`` returns x = 0.
    """
    nb = float(np.sqrt(b @ b))
    if nb == 0.0:
        return np.zeros_like(b), 0, OK
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x
    if np.sqrt(r @ r) <= tol * nb:
        return x, 0, OK
    z = dinv * r
    p = z.copy()
    rho = float(r @ z)
    for k in range(max_iter):
        q = A @ p
        sigma = float(p @ q)
        if not np.isfinite(sigma) or sigma <= 0.0:
            return x, k, ERR_BREAKDOWN
        alpha = rho / sigma
        x += alpha * p
        r -= alpha * q
        if np.sqrt(r @ r) <= tol * nb:
            return x, k + 1, OK
        z = dinv * r
        rho_new = float(r @ z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, max_iter, NOT_CONVERGED


def _check_system(sysm, solve_labels):
    if np.any(sysm.diag <= 0.0):
        raise OracleError(ERR_SINGULAR, "zero diagonal on an unknown voxel")
    present = set(np.unique(sysm.labels[sysm.M]).tolist())
    for s in solve_labels:
        if s not in present:
            raise OracleError(ERR_NO_SEEDS, f"label {s} has no seed")


def random_walker(g, labels, K, beta, method="pcg", tol=1e-6, max_iter=20000, w_eps=0.0,
                  x0=None, solve_labels=None, return_info=False):
    """Probability maps of the labels (every label solved independently).

    method: "pcg" (step-by-step Jacobi-PCG, same stopping rule as the GPU),
    "direct" (sparse LU), or "dense" (numpy.linalg.solve, tiny grids only).
    x0: optional initial guesses, [len(solve_labels)][grid] (default 0 on U).
    Returns x[len(solve_labels)][nz][ny][nx] (float64).
    """
    g = np.asarray(g, dtype=np.float64)
    sysm = DirichletSystem(g, labels, beta, w_eps, K)
    solve_labels = list(range(1, K + 1)) if solve_labels is None else list(solve_labels)
    _check_system(sysm, solve_labels)
    out = np.empty((len(solve_labels),) + g.shape)
    info = []
    if method == "dense":
        LUd = sysm.LU.toarray()
    elif method == "direct":
        lu = spla.splu(sysm.LU.tocsc())
    dinv = 1.0 / sysm.diag
    for k, s in enumerate(solve_labels):
        b = sysm.rhs(s)
        if method == "dense":
            xU = np.linalg.solve(LUd, b)
            it, st = 0, OK
        elif method == "direct":
            xU = lu.solve(b)
            it, st = 0, OK
        else:
            x0U = np.zeros(sysm.U.size) if x0 is None else np.asarray(x0[k]).ravel()[sysm.U]
            xU, it, st = pcg_jacobi(sysm.LU, b, dinv, x0U, tol, max_iter)
            if st < 0:
                raise OracleError(st, f"label {s}: PCG failed")
        nb = np.linalg.norm(b)
        rel = np.linalg.norm(b - sysm.LU @ xU) / nb if nb > 0 else 0.0
        info.append(dict(label=s, iters=it, status=st, rel_residual=rel))
        out[k] = sysm.full(s, xU)
    return (out, info) if return_info else out


def argmax_labels(prob):
    """1-based label of the largest probability; ties go to the lowest label."""
    return (np.argmax(prob, axis=0) + 1).astype(np.uint8)


# --------------------------------------------------------------------------
# matrix-vector building blocks used by kernel-level parity tests
# --------------------------------------------------------------------------

def operator_LU(g, labels, beta, w_eps=0.0):
    """(L_U as CSR, U index array) for SpMV parity: q_U = L_U p_U, zero on M."""
    sysm = DirichletSystem(np.asarray(g, dtype=np.float64), labels, beta, w_eps)
    return sysm.LU, sysm.U


def degrees(g, beta, w_eps=0.0):
    """d_i = sum of w_ij over all in-volume neighbours (the Laplacian diagonal)."""
    g = np.asarray(g, dtype=np.float64)
    L = laplacian(g.shape, edge_weights(g, beta, w_eps))
    return L.diagonal().reshape(g.shape)


# --------------------------------------------------------------------------
# hierarchy: levels, coarse seeds, upsampling, bricks
# --------------------------------------------------------------------------

def downsample_mean(a):
    """One LOD step: each coarse voxel is the mean of its (up to) 2x2x2 fine voxels.

    Coarse size is ceil(n / 2) per axis; at an odd far edge the box averages
    only the voxels that exist.
    """
    a = np.asarray(a, dtype=np.float64)
    nz, ny, nx = a.shape
    cz, cy, cx = (nz + 1) // 2, (ny + 1) // 2, (nx + 1) // 2
    s = np.zeros((cz, cy, cx))
    c = np.zeros((cz, cy, cx))
    for dz in range(2):
        for dy in range(2):
            for dx in range(2):
                sub = a[dz::2, dy::2, dx::2]
                s[:sub.shape[0], :sub.shape[1], :sub.shape[2]] += sub
                c[:sub.shape[0], :sub.shape[1], :sub.shape[2]] += 1
    return s / c


def coarse_seeds(labels):
    """One LOD step of the seed map: a coarse voxel takes label s when its
    (up to) 2x2x2 fine block holds at least one seed of s and none of another
    label; blocks with conflicting labels stay unseeded."""
    lab = np.asarray(labels)
    nz, ny, nx = lab.shape
    cz, cy, cx = (nz + 1) // 2, (ny + 1) // 2, (nx + 1) // 2
    K = int(lab.max()) if lab.size else 0
    present = np.zeros((K + 1, cz, cy, cx), dtype=bool)
    for dz in range(2):
        for dy in range(2):
            for dx in range(2):
                sub = lab[dz::2, dy::2, dx::2]
                for s in range(1, K + 1):
                    present[s, :sub.shape[0], :sub.shape[1], :sub.shape[2]] |= (sub == s)
    count = present[1:].sum(axis=0)
    out = np.zeros((cz, cy, cx), dtype=np.uint8)
    for s in range(1, K + 1):
        out[(count == 1) & present[s]] = s
    return out


def upsample_coords(n_fine, n_coarse, f):
    """Cell-centred fine -> coarse coordinate u = (i + 0.5)/f - 0.5, clamped."""
    u = (np.arange(n_fine, dtype=np.float64) + 0.5) / f - 0.5
    return np.clip(u, 0.0, n_coarse - 1)


def upsample_trilinear(coarse, fine_shape, f, region=None):
    """Trilinear, cell-centred, edge-clamped upsampling of a coarse field.

    region = (origin, size) restricts the output to a box of the fine grid
    (the box may extend outside the volume: those voxels are left NaN).
    """
    coarse = np.asarray(coarse, dtype=np.float64)
    nzc, nyc, nxc = coarse.shape
    if region is None:
        origin, size = (0, 0, 0), fine_shape
    else:
        origin, size = region

    def axis(o, s, n_f, n_c):
        i = np.arange(o, o + s)
        ok = (i >= 0) & (i < n_f)
        u = (i + 0.5) / f - 0.5
        u = np.clip(u, 0.0, n_c - 1)
        i0 = np.floor(u).astype(np.int64)
        i0 = np.minimum(i0, n_c - 1)
        i1 = np.minimum(i0 + 1, n_c - 1)
        t = u - i0
        return i0, i1, t, ok

    z0, z1, tz, okz = axis(origin[0], size[0], fine_shape[0], nzc)
    y0, y1, ty, oky = axis(origin[1], size[1], fine_shape[1], nyc)
    x0, x1, tx, okx = axis(origin[2], size[2], fine_shape[2], nxc)
    out = np.zeros(tuple(size))
    for zi, wz in ((z0, 1 - tz), (z1, tz)):
        for yi, wy in ((y0, 1 - ty), (y1, ty)):
            for xi, wx in ((x0, 1 - tx), (x1, tx)):
                out += (wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
                        * coarse[np.ix_(zi, yi, xi)])
    ok = okz[:, None, None] & oky[None, :, None] & okx[None, None, :]
    out[~ok] = np.nan
    return out


def brick_grid(shape, brick, offset):
    """Tile a volume into bricks on a regular grid shifted by ``offset``.

    Per axis the first brick spans [0, offset) (when offset > 0), then full
    bricks of ``brick`` voxels, then the remainder.  Returns a list of
    (origin_zyx, size_zyx) in z-major order.
    """
    def cuts(n, b, o):
        edges = [0]
        if o > 0:
            edges.append(min(o, n))
        while edges[-1] < n:
            edges.append(min(edges[-1] + b, n))
        return [(edges[k], edges[k + 1] - edges[k]) for k in range(len(edges) - 1)]

    out = []
    for oz, sz in cuts(shape[0], brick[0], offset[0]):
        for oy, sy in cuts(shape[1], brick[1], offset[1]):
            for ox, sx in cuts(shape[2], brick[2], offset[2]):
                out.append(((oz, oy, ox), (sz, sy, sx)))
    return out


def _shell_mask(shape, origin, size):
    """Voxels outside the box that share a face with it (6-connectivity)."""
    nz, ny, nx = shape
    o = np.array(origin)
    s = np.array(size)
    lo = np.maximum(o - 1, 0)
    hi = np.minimum(o + s + 1, [nz, ny, nx])
    zz, yy, xx = np.meshgrid(np.arange(lo[0], hi[0]), np.arange(lo[1], hi[1]),
                             np.arange(lo[2], hi[2]), indexing="ij")
    inside = [(a >= o[k]) & (a < o[k] + s[k]) for k, a in enumerate((zz, yy, xx))]
    n_out = sum((~m).astype(np.int64) for m in inside)
    shell = n_out == 1
    return zz[shell], yy[shell], xx[shell]


def classify_brick(P_frame, labels, shape, origin, size, lo_thr=0.02, hi_thr=0.98):
    """Activity of one brick.

    ``P_frame`` holds the upsampled coarse probabilities [K][sz+2][sy+2][sx+2]
    over the brick and a one-voxel frame (values outside the volume are
    ignored).  Active iff some voxel of the brick or of its face shell has some
    label with lo_thr < p < hi_thr (strict), or a seed inside the brick has a
    label other than the argmax (lowest label on ties) of the upsampled
    probabilities at that voxel.
    """
    o = np.array(origin)
    s = np.array(size)
    inner = P_frame[:, 1:-1, 1:-1, 1:-1]
    if ((inner > lo_thr) & (inner < hi_thr)).any():
        return True
    zz, yy, xx = _shell_mask(shape, origin, size)
    if zz.size:
        ps = P_frame[:, zz - o[0] + 1, yy - o[1] + 1, xx - o[2] + 1]
        if ((ps > lo_thr) & (ps < hi_thr)).any():
            return True
    lab = np.asarray(labels)[o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]]
    seeded = lab > 0
    if seeded.any():
        am = np.argmax(inner, axis=0) + 1
        if np.any(am[seeded] != lab[seeded]):
            return True
    return False


def solve_brick(g, labels, origin, size, shell_value, x0_box, beta, tol=1e-6,
                max_iter=20000, solve_labels=None, w_eps=0.0, method="pcg"):
    """Random walker restricted to one brick with Dirichlet data on its shell.

    Unknowns: unseeded voxels of the brick.  Dirichlet voxels: seeds inside
    the brick ([label = s]) and every in-volume face neighbour outside it (its
    seed value if seeded, else ``shell_value[s](z, y, x)``).  Weights use the
    full-resolution g at both ends, so the brick operator is the global
    Laplacian restricted to the brick.  Returns x[len(solve_labels)][box]
    and per-label info dicts.
    """
    g = np.asarray(g, dtype=np.float64)
    shape = g.shape
    o = np.array(origin)
    s = np.array(size)
    lo = np.maximum(o - 1, 0)
    hi = np.minimum(o + s + 1, shape)
    gb = g[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
    lb = np.asarray(labels)[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
    # local box = brick + (in-volume) one-voxel frame; frame voxels that are
    # not face neighbours of the brick are dropped from the graph entirely.
    bshape = gb.shape
    zz, yy, xx = np.meshgrid(np.arange(lo[0], hi[0]), np.arange(lo[1], hi[1]),
                             np.arange(lo[2], hi[2]), indexing="ij")
    inside = ((zz >= o[0]) & (zz < o[0] + s[0]) & (yy >= o[1]) & (yy < o[1] + s[1])
              & (xx >= o[2]) & (xx < o[2] + s[2]))
    n_out = (((zz < o[0]) | (zz >= o[0] + s[0])).astype(int)
             + ((yy < o[1]) | (yy >= o[1] + s[1])).astype(int)
             + ((xx < o[2]) | (xx >= o[2] + s[2])).astype(int))
    shell = n_out == 1
    edges = grid_edges(bshape)
    ei, ej, _ = edges
    keep_node = (inside | shell).ravel()
    ins = inside.ravel()
    # keep edges with at least one endpoint inside the brick and both in the graph
    keep = keep_node[ei] & keep_node[ej] & (ins[ei] | ins[ej])
    edges = (ei[keep], ej[keep], None)
    w = edge_weights(gb, beta, w_eps, edges)
    L = laplacian(bshape, w, edges)
    flat_lab = lb.ravel()
    U = np.flatnonzero(ins & (flat_lab == 0))
    Mi = np.flatnonzero(ins & (flat_lab > 0))
    Sh = np.flatnonzero(shell.ravel())
    LU = L[U][:, U].tocsr()
    if LU.shape[0] and np.any(LU.diagonal() <= 0):
        raise OracleError(ERR_SINGULAR, "zero diagonal in brick")
    dinv = 1.0 / LU.diagonal() if LU.shape[0] else np.zeros(0)
    Dset = np.concatenate([Mi, Sh])
    B = L[U][:, Dset].tocsr()
    K = int(np.asarray(labels).max())
    solve_labels = list(range(1, K + 1)) if solve_labels is None else list(solve_labels)
    sh_z, sh_y, sh_x = zz.ravel()[Sh], yy.ravel()[Sh], xx.ravel()[Sh]
    # map from brick-local coordinates into the box
    b_idx = np.flatnonzero(ins)
    out = np.empty((len(solve_labels),) + tuple(s))
    info = []
    for k, lab in enumerate(solve_labels):
        mvals = np.empty(Dset.size)
        mvals[:Mi.size] = (flat_lab[Mi] == lab)
        shl = flat_lab[Sh]
        sv = shell_value(lab, sh_z, sh_y, sh_x)
        mvals[Mi.size:] = np.where(shl > 0, (shl == lab).astype(np.float64), sv)
        b = -(B @ mvals)
        full = np.empty(lb.size)
        full[Mi] = flat_lab[Mi] == lab
        if U.size:
            x0U_box = np.asarray(x0_box[k]).ravel()
            # x0_box is over the brick; U indexes the frame box
            loc = np.zeros(lb.size)
            loc[b_idx] = x0U_box
            x0U = loc[U]
            if method == "direct" and U.size:
                xU, it, st = spla.spsolve(LU.tocsc(), b), 0, OK
            else:
                xU, it, st = pcg_jacobi(LU, b, dinv, x0U, tol, max_iter)
            if st < 0:
                raise OracleError(st, "brick PCG failed")
            full[U] = xU
        else:
            it, st = 0, OK
        out[k] = full[b_idx].reshape(tuple(s))
        info.append(dict(label=lab, iters=it, status=st))
    return out, info


def hierarchical_rw(g0, labels0, K, beta, levels=2, brick=(64, 64, 64), offset=(0, 0, 0),
                    tol=1e-6, max_iter=20000, lo_thr=0.02, hi_thr=0.98, coarse_method="pcg",
                    brick_method="pcg", coarse_solver=None, brick_solver=None):
    """Coarse-to-fine random walker, step by step.

    1. LOD levels 1..L by 2x2x2 means of g (beta unchanged across levels).
    2. Coarse seed maps by the conflict rule.
    3. The coarsest level is solved whole for every label.
    4. Level 0 is tiled into bricks; each brick's upsampled coarse
       probabilities (trilinear, cell-centred, f = 2^L) over brick and face
       shell decide its activity.
    5. Inactive bricks output the upsampled probabilities, seeds exact.
    6. Active bricks solve the brick problem with shell values from the
       upsampled coarse solution, x0 = the upsampled values.
    7. All labels are solved independently (their sum is checked, not imposed).

    Returns dict(prob=[K][grid], active=[bool per brick], bricks=list,
    coarse=[K][coarse grid], info=...).
    """
    g0 = np.asarray(g0, dtype=np.float64)
    gl, ll = g0, np.asarray(labels0)
    for _ in range(levels):
        gl = downsample_mean(gl)
        ll = coarse_seeds(ll)
    f = 2 ** levels
    if coarse_solver is not None:
        coarse = coarse_solver(gl, ll)
    else:
        coarse = random_walker(gl, ll, K, beta, method=coarse_method, tol=tol, max_iter=max_iter)
    shape = g0.shape

    def up(origin, size):
        return np.stack([upsample_trilinear(coarse[k], shape, f, (origin, size)) for k in range(K)])

    bricks = brick_grid(shape, brick, offset)
    prob = np.empty((K,) + shape)
    active = []
    infos = []
    for origin, size in bricks:
        o = np.array(origin)
        P_frame = up(tuple(o - 1), tuple(np.array(size) + 2))
        act = classify_brick(P_frame, labels0, shape, origin, size, lo_thr, hi_thr)
        active.append(act)
        sl = tuple(slice(a, a + b) for a, b in zip(origin, size))
        P = P_frame[:, 1:-1, 1:-1, 1:-1]
        if not act:
            lab = np.asarray(labels0)[sl]
            for k in range(K):
                blk = P[k].copy()
                seeded = lab > 0
                blk[seeded] = (lab[seeded] == k + 1)
                prob[k][sl] = blk
            continue

        def shell_value(lab, zz, yy, xx, P_frame=P_frame, o=o):
            return P_frame[lab - 1][zz - o[0] + 1, yy - o[1] + 1, xx - o[2] + 1]

        if brick_solver is not None:
            xb, info = brick_solver(origin, size, P_frame)
        else:
            xb, info = solve_brick(g0, labels0, origin, size, shell_value, P, beta, tol, max_iter,
                                   list(range(1, K + 1)), method=brick_method)
        for k in range(K):
            prob[k][sl] = xb[k]
        infos.append(info)
    return dict(prob=prob, active=np.array(active), bricks=bricks, coarse=coarse, info=infos,
                g_coarse=gl, labels_coarse=ll)


# --------------------------------------------------------------------------
# gradients (adjoint) and their independent checks
# --------------------------------------------------------------------------

def adjoint_gradient(g, labels, beta, label, dLdx_full, w_eps=0.0, x_full=None):
    """dL/dbeta and dL/dg for a loss L(x^label) via one adjoint solve.

    Adjoint: L_U lam = dL/dx_U (lam = 0 on M); per edge
    c_e = (lam_i - lam_j)(x_i - x_j) w_e; then
    dL/dbeta = sum_e c_e (g_i - g_j)^2 and
    dL/dg_i = sum_{e = (i, j)} 2 beta c_e (g_i - g_j).
    Solves are direct (exact), so this is the plain definition.
    """
    g = np.asarray(g, dtype=np.float64)
    sysm = DirichletSystem(g, labels, beta, w_eps)
    lu = spla.splu(sysm.LU.tocsc())
    if x_full is None:
        x_full = sysm.full(label, lu.solve(sysm.rhs(label)))
    xf = np.asarray(x_full).ravel()
    rhs = np.asarray(dLdx_full).ravel()[sysm.U]
    lam = np.zeros(g.size)
    lam[sysm.U] = lu.solve(rhs)
    i, j, _ = sysm.edges
    gf = g.ravel()
    dg = gf[i] - gf[j]
    c = (lam[i] - lam[j]) * (xf[i] - xf[j]) * sysm.w
    dbeta = float(np.sum(c * dg * dg))
    contrib = 2.0 * beta * c * dg
    dgr = np.zeros(g.size)
    np.add.at(dgr, i, contrib)
    np.add.at(dgr, j, -contrib)
    return dbeta, dgr.reshape(g.shape), lam.reshape(g.shape)


def seg_loss(x_fg, mask):
    """Sum over voxels of (x_fg - mask)^2 and its gradient 2 (x_fg - mask)."""
    d = np.asarray(x_fg) - np.asarray(mask, dtype=np.float64)
    return float(np.sum(d * d)), 2.0 * d


def complex_step_loss(g, labels, beta, label, mask, h=1e-30, d_beta=False, voxel=None):
    """Imaginary part of the loss after perturbing beta or g[voxel] by i*h,
    divided by h: the complex-step derivative (Squire & Trapp 1998), with a
    dense complex solve.  Tiny grids only."""
    g = np.asarray(g, dtype=np.complex128).copy()
    b_ = complex(beta)
    if d_beta:
        b_ += 1j * h
    if voxel is not None:
        g.flat[voxel] += 1j * h
    lab = np.asarray(labels).ravel()
    i, j, _ = grid_edges(g.shape)
    gf = g.ravel()
    diff = gf[i] - gf[j]
    w = np.exp(-b_ * diff * diff)
    n = g.size
    L = np.zeros((n, n), dtype=np.complex128)
    np.add.at(L, (i, j), -w)
    np.add.at(L, (j, i), -w)
    np.add.at(L, (i, i), w)
    np.add.at(L, (j, j), w)
    U = np.flatnonzero(lab == 0)
    M = np.flatnonzero(lab > 0)
    m = (lab[M] == label).astype(np.complex128)
    xU = np.linalg.solve(L[np.ix_(U, U)], -(L[np.ix_(U, M)] @ m))
    x = np.empty(n, dtype=np.complex128)
    x[M] = m
    x[U] = xU
    d = x - np.asarray(mask, dtype=np.float64).ravel()
    return float(np.imag(np.sum(d * d)) / h)


# --------------------------------------------------------------------------
# Monte-Carlo random walks (model semantics)
# --------------------------------------------------------------------------

def monte_carlo_walks(g, labels, beta, start_flat, n_walks, rng, max_steps=100000):
    """First-arrival label frequencies of walkers released at a voxel.

    Each step moves to a 6-neighbour with probability proportional to the
    edge weight; a walk ends at the first seeded voxel it reaches.
    Returns the frequency of each label 1..K.
    """
    g = np.asarray(g, dtype=np.float64)
    shape = g.shape
    nz, ny, nx = shape
    n = g.size
    lab = np.asarray(labels).ravel()
    K = int(lab.max())
    # neighbour table (n, 6) and weights
    idx = np.arange(n)
    z, y, x = idx // (ny * nx), (idx // nx) % ny, idx % nx
    nbr = np.full((n, 6), -1, dtype=np.int64)
    steps = [(0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)]
    for k, (dz, dy, dx) in enumerate(steps):
        zz, yy, xx = z + dz, y + dy, x + dx
        ok = (zz >= 0) & (zz < nz) & (yy >= 0) & (yy < ny) & (xx >= 0) & (xx < nx)
        nbr[ok, k] = (zz * ny + yy)[ok] * nx + xx[ok]
    gf = g.ravel()
    wn = np.where(nbr >= 0, np.exp(-beta * (gf[:, None] - gf[np.maximum(nbr, 0)]) ** 2), 0.0)
    cdf = np.cumsum(wn, axis=1)
    cdf /= cdf[:, -1:]
    pos = np.full(n_walks, start_flat, dtype=np.int64)
    alive = lab[pos] == 0
    result = np.where(alive, 0, lab[pos]).astype(np.int64)
    for _ in range(max_steps):
        if not alive.any():
            break
        a = np.flatnonzero(alive)
        u = rng.random(a.size)
        choice = (u[:, None] > cdf[pos[a]]).sum(axis=1)
        pos[a] = nbr[pos[a], choice]
        hit = lab[pos[a]] > 0
        result[a[hit]] = lab[pos[a[hit]]]
        alive[a[hit]] = False
    return np.array([(result == s).mean() for s in range(1, K + 1)])
