"""GPU adjoint gradients against the oracle's direct-solve adjoint, central
finite differences (float64 solves at tol 1e-12) and torch.autograd."""
import numpy as np
import pytest

from oracle import rw_oracle as O
from synth import random_case, sphere_case
from tests._helpers import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    from paper_2509_26213_amd import rw as m
    m.lib()
    return m


def test_adjoint_matches_oracle_direct(rw):
    c = random_case((9, 10, 11), K=2, seeds_per_label=8, beta=8.0, seed=5)
    g = O.case_g(c)
    mask = (np.random.default_rng(1).random(g.shape) > 0.5).astype(float)
    x = O.random_walker(g, c.labels, 2, 8.0, method="direct")[1]
    _, dLdx = O.seg_loss(x, mask)
    db_ref, dg_ref, _ = O.adjoint_gradient(g, c.labels, 8.0, 2, dLdx, x_full=x)
    prob = np.stack([1.0 - x, x])
    grad_prob = np.stack([np.zeros_like(x), dLdx])
    dg, db = rw.solve_backward(dev(g), dev(c.labels), 2, 8.0, dev(prob), dev(grad_prob),
                               tol=1e-13)
    db = float(db)
    assert abs(db - db_ref) <= 1e-8 * max(1.0, abs(db_ref))
    assert np.max(np.abs(host(dg) - dg_ref)) <= 1e-8 * max(1.0, np.max(np.abs(dg_ref)))


def test_autograd_three_labels(rw):
    import torch
    c = random_case((8, 9, 10), K=3, seeds_per_label=6, beta=6.0, seed=9)
    g = O.case_g(c)
    w = np.random.default_rng(2).standard_normal((3,) + g.shape)
    gt = dev(g).requires_grad_(True)
    beta = torch.tensor(6.0, dtype=torch.float64, device="cuda", requires_grad=True)
    prob = rw.random_walker(gt, beta, dev(c.labels), 3, tol=1e-13)
    loss = (prob * dev(w)).sum()
    loss.backward()
    # oracle: the same loss through the oracle's solves of labels 2, 3
    xs = O.random_walker(g, c.labels, 3, 6.0, method="direct")
    db_ref = 0.0
    dg_ref = np.zeros_like(g)
    for s in (2, 3):
        gs = w[s - 1] - w[0]
        db, dg, _ = O.adjoint_gradient(g, c.labels, 6.0, s, gs, x_full=xs[s - 1])
        db_ref += db
        dg_ref += dg
    assert abs(beta.grad.item() - db_ref) <= 1e-8 * max(1, abs(db_ref))
    assert np.max(np.abs(host(gt.grad) - dg_ref)) <= 1e-8 * max(1, np.max(np.abs(dg_ref)))


def test_sphere_gradients_vs_central_differences(rw):
    """Scaled differentiable case: 48^3 sphere, loss sum (x_fg - mask)^2,
    dL/dbeta and dL/dg on sampled voxels vs central differences of float64
    GPU solves at tol 1e-12 (x0 = 0)."""
    import torch
    c = sphere_case(n=48, radius=15, sigma=0.1, seed_radius=7, corner=6, n_seeds=300,
                    beta=120.0, seed=4)
    g = O.case_g(c)
    mask = c.truth.astype(np.float64)
    gd, lab, md = dev(g), dev(c.labels), dev(mask)

    def loss(gg, b):
        prob, _ = rw.solve(gg, lab, 2, b, tol=1e-12, precision="fp64", lo=0.0, hi=1.0,
                           argmax=False)
        return float(((prob[1] - md) ** 2).sum())

    prob, _ = rw.solve(gd, lab, 2, 120.0, tol=1e-12, precision="fp64", lo=0.0, hi=1.0)
    grad_prob = torch.stack([torch.zeros_like(md), 2 * (prob[1] - md)])
    dg, db = rw.solve_backward(gd, lab, 2, 120.0, prob, grad_prob, tol=1e-12)
    db = float(db)
    h = 1e-4
    fd_b = (loss(gd, 120.0 + h) - loss(gd, 120.0 - h)) / (2 * h)
    assert abs(fd_b - db) <= 1e-4 * max(abs(fd_b), 1e-12), (fd_b, db)
    rng = np.random.default_rng(0)
    dist = np.sqrt(((np.indices(g.shape) - (g.shape[0] - 1) / 2) ** 2).sum(0))
    near = np.flatnonzero((np.abs(dist - 15) <= 2).ravel() & (c.labels.ravel() == 0))
    pick = np.concatenate([rng.choice(near, 6, replace=False),
                           rng.choice(np.flatnonzero(c.labels.ravel() == 0), 4, replace=False)])
    fds, ads = [], []
    hg = 1e-3
    for v in pick:
        gp = gd.clone().view(-1)
        gm = gd.clone().view(-1)
        gp[v] += hg
        gm[v] -= hg
        fds.append((loss(gp.view(g.shape), 120.0) - loss(gm.view(g.shape), 120.0)) / (2 * hg))
        ads.append(float(dg.view(-1)[v]))
    fds, ads = np.array(fds), np.array(ads)
    scale = max(np.sqrt(np.mean(fds ** 2)), 1e-12)
    assert np.all(np.abs(ads - fds) <= 1e-3 * np.maximum(np.abs(fds), scale)), (ads, fds)
