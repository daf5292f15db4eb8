"""Pins of the CPU oracle against what mathematics fixes (no GPU).

Each test names the property of the random-walker Dirichlet problem (the
paper's Sec. III-A operator) or of Jacobi-PCG that it checks.
"""
import os

import numpy as np
import pytest

from oracle import rw_oracle as O
from synth import random_case, sphere_case, blob_case

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random(shape, K, seeds, beta, seed):
    c = random_case(shape, K=K, seeds_per_label=seeds, beta=beta, seed=seed)
    return O.case_g(c), c.labels, c


# ---------------------------------------------------------------- exact fixture

def _read_golden(name):
    meta, rows = {}, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("# "):
                parts = line[2:].split()
                if parts and parts[0] in ("shape", "beta", "g", "labels"):
                    meta[parts[0]] = parts[1:]
                continue
            rows.append([float(v) for v in line.split()])
    return meta, np.array(rows)


def test_exact_rational_fixture_dense_and_pcg():
    meta, rows = _read_golden("rw_exact_3x3x3.txt")
    shape = tuple(int(v) for v in meta["shape"])
    g = np.array([float(v) for v in meta["g"]]).reshape(shape)
    lab = np.array([int(v) for v in meta["labels"]], dtype=np.uint8).reshape(shape)
    beta = float(meta["beta"][0])
    ref = rows[:, 1:].T.reshape((3,) + shape)
    xd = O.random_walker(g, lab, 3, beta, method="dense")
    xp = O.random_walker(g, lab, 3, beta, method="pcg", tol=1e-14)
    assert np.max(np.abs(xd - ref)) < 1e-14
    assert np.max(np.abs(xp - ref)) < 1e-12


def test_exact_rational_fixture_c_oracle(c_oracle):
    meta, rows = _read_golden("rw_exact_3x3x3.txt")
    shape = tuple(int(v) for v in meta["shape"])
    g = np.array([float(v) for v in meta["g"]]).reshape(shape)
    lab = np.array([int(v) for v in meta["labels"]], dtype=np.uint8).reshape(shape)
    ref = rows[:, 1:].T.reshape((3,) + shape)
    xc = c_oracle.random_walker(g, lab, 3, float(meta["beta"][0]), tol=1e-14)
    assert np.max(np.abs(xc - ref)) < 1e-12


# ---------------------------------------------------------------- library routines

@pytest.mark.parametrize("seed,K", [(0, 2), (1, 3), (2, 4)])
def test_pcg_matches_dense_direct(seed, K):
    g, lab, c = _random((6, 5, 7), K, 3, 8.0, seed)
    xd = O.random_walker(g, lab, K, 8.0, method="dense")
    xp = O.random_walker(g, lab, K, 8.0, method="pcg", tol=1e-13)
    assert np.max(np.abs(xd - xp)) < 1e-10


def test_sparse_direct_matches_dense():
    g, lab, _ = _random((8, 8, 8), 3, 4, 20.0, 7)
    xd = O.random_walker(g, lab, 3, 20.0, method="dense")
    xs = O.random_walker(g, lab, 3, 20.0, method="direct")
    assert np.max(np.abs(xd - xs)) < 1e-12


def test_assembled_laplacian_matches_scipy_csgraph():
    from scipy.sparse.csgraph import laplacian as cs_lap
    import scipy.sparse as sp
    g, _, _ = _random((4, 5, 6), 2, 2, 3.0, 3)
    i, j, _ = O.grid_edges(g.shape)
    w = O.edge_weights(g, 3.0)
    n = g.size
    W = sp.coo_matrix((np.r_[w, w], (np.r_[i, j], np.r_[j, i])), shape=(n, n)).toarray()
    L = O.laplacian(g.shape, w).toarray()
    assert np.allclose(L, cs_lap(W), atol=1e-15)
    # every voxel's degree = sum of its in-volume neighbour weights
    assert np.allclose(O.degrees(g, 3.0).ravel(), W.sum(1))


def test_edge_count_and_weight_layout():
    shape = (3, 4, 5)
    i, j, a = O.grid_edges(shape)
    nz, ny, nx = shape
    assert i.size == nz * ny * (nx - 1) + nz * (ny - 1) * nx + (nz - 1) * ny * nx
    g = np.random.default_rng(0).random(shape)
    w3 = O.weights_grid(g, 2.0)
    assert np.all(w3[0][:, :, -1] == 0) and np.all(w3[1][:, -1, :] == 0) and np.all(w3[2][-1] == 0)
    z, y, x = 1, 2, 3
    assert np.isclose(w3[0][z, y, x], np.exp(-2.0 * (g[z, y, x + 1] - g[z, y, x]) ** 2))
    assert np.isclose(w3[2][z, y, x], np.exp(-2.0 * (g[z + 1, y, x] - g[z, y, x]) ** 2))


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [5, 17])
def test_linear_ramp_constant_image(n, c_oracle):
    """Constant image, fg plane at x=0, bg plane at x=n-1: x_fg = 1 - i/(n-1)."""
    shape = (4, 3, n)
    g = np.full(shape, 0.37)
    lab = np.zeros(shape, dtype=np.uint8)
    lab[:, :, 0] = 2
    lab[:, :, -1] = 1
    ramp = 1.0 - np.arange(n) / (n - 1)
    for x in (O.random_walker(g, lab, 2, 50.0, method="pcg", tol=1e-13)[1],
              c_oracle.random_walker(g, lab, 2, 50.0, tol=1e-13)[1]):
        assert np.max(np.abs(x - ramp[None, None, :])) < 1e-11


def test_resistor_divider_closed_form(c_oracle):
    """Image varying only along x: series resistors R_k = exp(beta dg_k^2)."""
    n, beta = 12, 30.0
    prof = np.random.default_rng(5).random(n)
    g = np.broadcast_to(prof, (3, 4, n)).copy()
    lab = np.zeros(g.shape, dtype=np.uint8)
    lab[:, :, 0] = 2
    lab[:, :, -1] = 1
    R = np.exp(beta * np.diff(prof) ** 2)
    expect = np.array([R[i:].sum() / R.sum() for i in range(n)])
    for x in (O.random_walker(g, lab, 2, beta, method="dense")[1],
              O.random_walker(g, lab, 2, beta, method="pcg", tol=1e-14)[1],
              c_oracle.random_walker(g, lab, 2, beta, tol=1e-14)[1]):
        assert np.max(np.abs(x - expect[None, None, :])) < 1e-11


def test_no_seed_label_gives_zero_and_single_label_gives_one():
    g, lab, _ = _random((5, 5, 5), 1, 4, 10.0, 2)
    x = O.random_walker(g, lab, 1, 10.0, method="pcg", tol=1e-12)
    assert np.allclose(x[0], 1.0, atol=1e-10)


# ---------------------------------------------------------------- invariants

def test_maximum_principle_and_sum_to_one():
    g, lab, _ = _random((9, 8, 7), 3, 5, 25.0, 11)
    tol = 1e-8
    x = O.random_walker(g, lab, 3, 25.0, method="pcg", tol=tol)
    assert x.min() >= -10 * tol and x.max() <= 1 + 10 * tol
    assert np.max(np.abs(x.sum(0) - 1.0)) < 1e-6
    seeded = lab > 0
    for s in (1, 2, 3):
        assert np.all(x[s - 1][seeded] == (lab[seeded] == s))


def test_rhs_consistency_LU_ones_equals_sum_b():
    g, lab, _ = _random((6, 6, 6), 3, 3, 15.0, 4)
    sysm = O.DirichletSystem(g, lab, 15.0)
    lhs = sysm.LU @ np.ones(sysm.U.size)
    rhs = sum(sysm.rhs(s) for s in (1, 2, 3))
    # L_U 1 + B 1 = 0 (rows of L sum to zero) and sum_s m^s = 1 on M
    assert np.allclose(lhs, rhs, atol=1e-13)


def test_spmv_symmetric():
    g, lab, _ = _random((5, 6, 7), 2, 3, 12.0, 8)
    A, U = O.operator_LU(g, lab, 12.0)
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal(U.size), rng.standard_normal(U.size)
    assert np.isclose(v @ (A @ u), u @ (A @ v), rtol=1e-13)


def test_beta_zero_image_independent():
    _, lab, _ = _random((6, 6, 6), 2, 3, 0.0, 9)
    g1 = np.random.default_rng(1).random(lab.shape)
    g2 = np.random.default_rng(2).random(lab.shape)
    x1 = O.random_walker(g1, lab, 2, 0.0, method="dense")
    x2 = O.random_walker(g2, lab, 2, 0.0, method="dense")
    assert np.max(np.abs(x1 - x2)) < 1e-13


@pytest.mark.parametrize("perm,flip", [((2, 1, 0), None), ((1, 0, 2), 0), ((0, 2, 1), 2)])
def test_axis_permutation_and_mirror_equivariance(perm, flip):
    g, lab, _ = _random((5, 6, 7), 3, 3, 9.0, 12)
    x = O.random_walker(g, lab, 3, 9.0, method="dense")

    def T(a):
        a = np.transpose(a, perm)
        return np.flip(a, flip) if flip is not None else a

    xt = O.random_walker(np.ascontiguousarray(T(g)), np.ascontiguousarray(T(lab)), 3, 9.0,
                         method="dense")
    for k in range(3):
        assert np.max(np.abs(xt[k] - T(x[k]))) < 1e-12


# ---------------------------------------------------------------- solver semantics

def test_pcg_stopping_rule_and_same_x0():
    g, lab, _ = _random((7, 7, 7), 2, 4, 30.0, 13)
    sysm = O.DirichletSystem(g, lab, 30.0)
    b = sysm.rhs(2)
    dinv = 1.0 / sysm.diag
    x, it, st = O.pcg_jacobi(sysm.LU, b, dinv, np.zeros(b.size), 1e-6, 10000)
    assert st == O.OK
    # the recursive residual met the rule; the true residual agrees closely
    assert np.linalg.norm(b - sysm.LU @ x) <= 1.01e-6 * np.linalg.norm(b)
    # one fewer iteration does not meet it
    x1, it1, st1 = O.pcg_jacobi(sysm.LU, b, dinv, np.zeros(b.size), 1e-6, it - 1)
    assert st1 == O.NOT_CONVERGED and it1 == it - 1
    assert np.linalg.norm(b - sysm.LU @ x1) > 1e-6 * np.linalg.norm(b)


def test_failure_statuses():
    g, lab, _ = _random((4, 4, 4), 2, 2, 5.0, 1)
    with pytest.raises(O.OracleError) as e:
        O.random_walker(g, np.zeros_like(lab), 2, 5.0)
    assert e.value.status == O.ERR_NO_SEEDS
    lab2 = lab.copy()
    lab2[lab2 == 2] = 0
    with pytest.raises(O.OracleError) as e:
        O.random_walker(g, lab2, 2, 5.0)
    assert e.value.status == O.ERR_NO_SEEDS
    # one unseeded voxel whose six weights all underflow to 0 in float64
    gs = np.zeros((3, 3, 3))
    gs[1, 1, 1] = 1.0
    ls = np.ones((3, 3, 3), dtype=np.uint8)
    ls[1, 1, 1] = 0
    ls[0, 0, 0] = 2
    with pytest.raises(O.OracleError) as e:
        O.random_walker(gs, ls, 2, 1000.0)
    assert e.value.status == O.ERR_SINGULAR


def test_c_oracle_statuses(c_oracle):
    gs = np.zeros((3, 3, 3))
    gs[1, 1, 1] = 1.0
    ls = np.ones((3, 3, 3), dtype=np.uint8)
    ls[1, 1, 1] = 0
    _, _, st, _ = c_oracle.solve_box(gs, ls, 1, 1000.0)
    assert st == -3
    g, lab, _ = _random((6, 6, 6), 2, 3, 20.0, 3)
    _, it, st, _ = c_oracle.solve_box(g, lab, 2, 20.0, tol=1e-10, max_iter=2)
    assert st == 1 and it == 2


# ---------------------------------------------------------------- brute force

@pytest.mark.slow
def test_monte_carlo_walks_agree():
    """First-arrival label frequencies of weighted random walks = x (model semantics)."""
    g, lab, _ = _random((4, 4, 4), 2, 3, 4.0, 21)
    x = O.random_walker(g, lab, 2, 4.0, method="dense")
    rng = np.random.default_rng(0)
    U = np.flatnonzero(lab.ravel() == 0)
    n_walks = 40000
    for v in U[:6]:
        freq = O.monte_carlo_walks(g, lab, 4.0, int(v), n_walks, rng)
        p = x[:, :, :, :].reshape(2, -1)[:, v]
        se = np.sqrt(p * (1 - p) / n_walks) + 1e-12
        assert np.all(np.abs(freq - p) <= 5 * se + 1e-3), (v, freq, p)


# ---------------------------------------------------------------- C oracle == Python oracle

@pytest.mark.parametrize("seed", [0, 1])
def test_c_oracle_matches_python_oracle(seed, c_oracle):
    c = blob_case(shape=(20, 24, 28), n_blobs=4, K=3, seeds_per_label=15, sigma=0.08,
                  rmin=3, rmax=8, seed=seed)
    g = O.case_g(c)
    xp, ip = O.random_walker(g, c.labels, 3, 150.0, method="pcg", tol=1e-6, return_info=True)
    xc, ic = c_oracle.random_walker(g, c.labels, 3, 150.0, tol=1e-6, return_info=True)
    assert [a["iters"] for a in ip] == [a["iters"] for a in ic]
    assert np.max(np.abs(xp - xc)) < 1e-10


def test_c_oracle_weights_match_python(c_oracle):
    g = np.random.default_rng(3).random((5, 6, 7))
    w6 = c_oracle.box_weights(g, 7.0)
    w3 = O.weights_grid(g, 7.0)
    assert np.allclose(w6[0], w3[0], rtol=1e-14, atol=0)          # +x
    assert np.allclose(w6[2], w3[1], rtol=1e-14, atol=0)          # +y
    assert np.allclose(w6[4], w3[2], rtol=1e-14, atol=0)          # +z
    assert np.allclose(w6[1][:, :, 1:], w3[0][:, :, :-1], rtol=1e-14, atol=0)  # -x


def test_sphere_case_o_same_close_to_o_exact(c_oracle):
    """On the 64^3 sphere case the tolerance-stopped solve is within 1e-5 of
    a tol = 1e-12 solve, so max-abs 1e-5 parity is meaningful there."""
    c = sphere_case()
    g = O.case_g(c)
    xs = c_oracle.random_walker(g, c.labels, 2, c.beta, tol=1e-6)
    xe = c_oracle.random_walker(g, c.labels, 2, c.beta, tol=1e-12)
    assert np.max(np.abs(xs - xe)) < 1e-5
    assert np.max(np.abs(xe.sum(0) - 1)) < 1e-9


# ---------------------------------------------------------------- C oracle residual

def test_c_oracle_residual_hand_computed_3x3x3(c_oracle):
    """Constant image (all weights 1), fg seed at (0,0,0), bg seed at (2,2,2),
    x = 1/2 on every unknown: the residual b - A x = sum_j w (x_j - x_i) is
    +1/2 at the three face neighbours of the fg seed, -1/2 at those of the bg
    seed, 0 elsewhere, and b is 1 at the fg seed's neighbours: for label 2
    ||r|| / ||b|| = sqrt(6/4) / sqrt(3) = sqrt(1/2); for label 1 the same by
    symmetry.  A wrong sign of A x (b + A x) would give 3/2 at those voxels."""
    g = np.zeros((3, 3, 3))
    lab = np.zeros((3, 3, 3), dtype=np.uint8)
    lab[0, 0, 0] = 2
    lab[2, 2, 2] = 1
    x = np.full(g.shape, 0.5)
    for s in (1, 2):
        assert abs(c_oracle.residual(g, lab, s, 5.0, x) - np.sqrt(0.5)) < 1e-15


def _assembled_rel_residual(g, lab, s, beta, x):
    sysm = O.DirichletSystem(g, lab, beta)
    b = sysm.rhs(s)
    xU = np.asarray(x).ravel()[sysm.U]
    return np.linalg.norm(b - sysm.LU @ xU) / np.linalg.norm(b)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c_oracle_residual_matches_assembled(seed, c_oracle):
    """orc_residual against the assembled ||b - L_U x|| / ||b|| for random x
    on a ragged three-label blob volume (seed values in x are ignored)."""
    c = blob_case(shape=(11, 14, 19), n_blobs=3, K=3, seeds_per_label=6, sigma=0.08,
                  rmin=3, rmax=6, seed=seed)
    g = O.case_g(c)
    rng = np.random.default_rng(seed)
    x = rng.random(g.shape)
    for s in (1, 2, 3):
        ref = _assembled_rel_residual(g, c.labels, s, c.beta, x)
        got = c_oracle.residual(g, c.labels, s, c.beta, x)
        assert abs(got - ref) <= 1e-12 * ref, (s, got, ref)
    # seed values in x do not enter
    x2 = x.copy()
    x2[c.labels > 0] = 123.0
    assert c_oracle.residual(g, c.labels, 2, c.beta, x2) == c_oracle.residual(g, c.labels, 2,
                                                                               c.beta, x)


def test_c_oracle_residual_of_exact_solution_is_zero(c_oracle):
    """At the direct solution the residual is at rounding level, and one
    perturbed unknown raises it to the assembled value."""
    c = blob_case(shape=(10, 12, 15), n_blobs=3, K=3, seeds_per_label=6, sigma=0.08,
                  rmin=3, rmax=6, seed=4)
    g = O.case_g(c)
    x = O.random_walker(g, c.labels, 3, c.beta, method="direct")
    for s in (1, 2, 3):
        assert c_oracle.residual(g, c.labels, s, c.beta, x[s - 1]) < 1e-12
    xp = x[1].copy()
    v = int(np.flatnonzero(c.labels.ravel() == 0)[7])
    xp.flat[v] += 1e-3
    ref = _assembled_rel_residual(g, c.labels, 2, c.beta, xp)
    assert ref > 1e-6
    assert abs(c_oracle.residual(g, c.labels, 2, c.beta, xp) - ref) <= 1e-9 * ref
