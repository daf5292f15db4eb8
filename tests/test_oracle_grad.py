"""Pins of the oracle's adjoint gradient: complex step (Squire & Trapp 1998),
the closed-form resistor divider, and central differences."""
import numpy as np
import pytest

from oracle import rw_oracle as O
from synth import random_case


def _case(seed=3, shape=(4, 4, 5), beta=6.0):
    c = random_case(shape, K=2, seeds_per_label=3, beta=beta, seed=seed)
    g = O.case_g(c)
    mask = (np.random.default_rng(seed + 100).random(shape) > 0.5).astype(float)
    return g, c.labels, mask


def _loss_and_grad(g, lab, beta, mask):
    x = O.random_walker(g, lab, 2, beta, method="dense")[1]
    L, dLdx = O.seg_loss(x, mask)
    db, dg, _ = O.adjoint_gradient(g, lab, beta, 2, dLdx, x_full=x)
    return L, db, dg


@pytest.mark.parametrize("seed", [3, 4])
def test_adjoint_matches_complex_step(seed):
    beta = 6.0
    g, lab, mask = _case(seed, beta=beta)
    _, db, dg = _loss_and_grad(g, lab, beta, mask)
    cs_b = O.complex_step_loss(g, lab, beta, 2, mask, d_beta=True)
    assert abs(db - cs_b) <= 1e-10 * max(1.0, abs(cs_b))
    rng = np.random.default_rng(seed)
    vox = list(rng.choice(g.size, 6, replace=False)) + [int(np.flatnonzero(lab.ravel())[0])]
    for v in vox:
        cs = O.complex_step_loss(g, lab, beta, 2, mask, voxel=int(v))
        assert abs(dg.ravel()[v] - cs) <= 1e-10 * max(1.0, abs(cs)), v


def test_adjoint_matches_central_differences():
    beta = 6.0
    g, lab, mask = _case(5, beta=beta)
    _, db, dg = _loss_and_grad(g, lab, beta, mask)
    h = 1e-6
    Lp = _loss_and_grad(g, lab, beta + h, mask)[0]
    Lm = _loss_and_grad(g, lab, beta - h, mask)[0]
    assert abs((Lp - Lm) / (2 * h) - db) < 1e-6 * max(1, abs(db))
    v = 17
    gp, gm = g.copy(), g.copy()
    gp.flat[v] += h
    gm.flat[v] -= h
    fd = (_loss_and_grad(gp, lab, beta, mask)[0] - _loss_and_grad(gm, lab, beta, mask)[0]) / (2 * h)
    assert abs(fd - dg.flat[v]) < 1e-6 * max(1, abs(fd))


def test_resistor_divider_beta_derivative():
    """d/dbeta of the closed-form divider, loss = sum over voxels of x_fg."""
    n, beta = 9, 20.0
    prof = np.random.default_rng(2).random(n)
    g = np.broadcast_to(prof, (2, 2, n)).copy()
    lab = np.zeros(g.shape, dtype=np.uint8)
    lab[:, :, 0] = 2
    lab[:, :, -1] = 1
    d2 = np.diff(prof) ** 2
    R = np.exp(beta * d2)
    dR = d2 * R
    S, dS = R.sum(), dR.sum()
    dx = np.array([(dR[i:].sum() * S - R[i:].sum() * dS) / S ** 2 for i in range(n)])
    expect = 4 * dx.sum()          # four identical rows; loss = sum x_fg
    x = O.random_walker(g, lab, 2, beta, method="dense")[1]
    db, _, _ = O.adjoint_gradient(g, lab, beta, 2, np.ones(g.shape), x_full=x)
    assert abs(db - expect) < 1e-10 * max(1, abs(expect))


# ---------------------------------------------------------------- C oracle adjoint

@pytest.mark.parametrize("seed", [3, 4])
def test_c_oracle_adjoint_matches_complex_step(seed, c_oracle):
    """The C oracle's adjoint (its own Jacobi-PCG on the adjoint system, then
    the edge sums) gives the complex-step derivatives of the loss."""
    beta = 6.0
    g, lab, mask = _case(seed, beta=beta)
    x = O.random_walker(g, lab, 2, beta, method="dense")[1]
    _, dLdx = O.seg_loss(x, mask)
    db, dg, lam, it, st = c_oracle.adjoint_gradient(g, lab, beta, x, dLdx, tol=1e-14)
    assert st == 0 and it > 0
    assert np.all(lam[lab > 0] == 0.0)
    cs_b = O.complex_step_loss(g, lab, beta, 2, mask, d_beta=True)
    assert abs(db - cs_b) <= 1e-10 * max(1.0, abs(cs_b))
    rng = np.random.default_rng(seed)
    vox = list(rng.choice(g.size, 6, replace=False)) + [int(np.flatnonzero(lab.ravel())[0])]
    for v in vox:
        cs = O.complex_step_loss(g, lab, beta, 2, mask, voxel=int(v))
        assert abs(dg.ravel()[v] - cs) <= 1e-10 * max(1.0, abs(cs)), v


def test_c_oracle_adjoint_matches_python_on_a_blob_case(c_oracle):
    """Against the assembled-matrix adjoint (sparse direct solves) on a
    ragged three-label blob volume, label 3."""
    from synth import blob_case
    c = blob_case(shape=(13, 17, 22), n_blobs=3, K=3, seeds_per_label=8, sigma=0.08,
                  rmin=3, rmax=6, seed=9)
    g = O.case_g(c)
    x = O.random_walker(g, c.labels, 3, c.beta, method="direct")[2]
    mask = (np.random.default_rng(1).random(g.shape) > 0.5).astype(float)
    _, dLdx = O.seg_loss(x, mask)
    db_p, dg_p, lam_p = O.adjoint_gradient(g, c.labels, c.beta, 3, dLdx, x_full=x)
    db_c, dg_c, lam_c, _, st = c_oracle.adjoint_gradient(g, c.labels, c.beta, x, dLdx, tol=1e-13)
    assert st == 0
    assert abs(db_c - db_p) <= 1e-9 * max(1.0, abs(db_p))
    assert np.max(np.abs(dg_c - dg_p)) <= 1e-9 * max(1.0, np.max(np.abs(dg_p)))
    assert np.max(np.abs(lam_c - lam_p)) <= 1e-9 * max(1.0, np.max(np.abs(lam_p)))


def test_c_oracle_adjoint_resistor_divider(c_oracle):
    """d/dbeta of the closed-form divider (loss = sum of x_fg) from the C oracle."""
    n, beta = 9, 20.0
    prof = np.random.default_rng(2).random(n)
    g = np.broadcast_to(prof, (2, 2, n)).copy()
    lab = np.zeros(g.shape, dtype=np.uint8)
    lab[:, :, 0] = 2
    lab[:, :, -1] = 1
    d2 = np.diff(prof) ** 2
    R = np.exp(beta * d2)
    dR = d2 * R
    S, dS = R.sum(), dR.sum()
    dx = np.array([(dR[i:].sum() * S - R[i:].sum() * dS) / S ** 2 for i in range(n)])
    expect = 4 * dx.sum()
    x = np.broadcast_to(np.array([R[i:].sum() / S for i in range(n)]), g.shape).copy()
    db, _, _, _, st = c_oracle.adjoint_gradient(g, lab, beta, x, np.ones(g.shape), tol=1e-14)
    assert st == 0
    assert abs(db - expect) < 1e-10 * max(1, abs(expect))
