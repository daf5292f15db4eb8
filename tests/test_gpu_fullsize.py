"""Parity at the full sizes of the benchmark configurations, through
properties the CPU oracle can check at any size: its own float64 residual of
the GPU's solutions, mixed vs float64 agreement, partition of unity, exact
seeds; and finite differences of the 128^3 differentiable case."""
import numpy as np
import pytest

from synth import blob_case, sphere_case
from tests._helpers import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    from paper_2509_26213_amd import rw as m
    m.lib()
    return m


def test_blob512_fullsize_properties(rw):
    import torch
    from oracle import c_oracle, rw_oracle
    c = blob_case(shape=(512, 512, 512), n_blobs=32, K=3, seeds_per_label=1000, sigma=0.08,
                  bg=0.2, rmin=10.0, rmax=60.0, beta=150.0, seed=2, dtype="f32")
    vol, lab = dev(c.vol), dev(c.labels)
    lo, hi = rw.minmax(vol)
    assert (lo, hi) == (float(c.vol.min()), float(c.vol.max()))
    p64, a64, s64 = rw.solve(vol, lab, 3, c.beta, tol=1e-6, precision="fp64", lo=lo, hi=hi,
                             return_stats=True)
    p32, a32, s32 = rw.solve(vol, lab, 3, c.beta, tol=1e-6, precision="mixed", lo=lo, hi=hi,
                             return_stats=True)
    assert s64["status"] == 0 and s32["status"] == 0
    d = (p32.double() - p64).abs().max().item()
    assert d <= 1e-5, d
    # argmax identical wherever the float64 top-two gap is at least 1e-4
    top2 = torch.topk(p64, 2, dim=0).values
    clear = (top2[0] - top2[1]) >= 1e-4
    bad = int(((a32 != a64) & clear).sum())
    assert bad == 0, bad
    assert torch.equal(a64, (p64.argmax(0) + 1).to(torch.uint8))
    del top2, clear, p32, a32
    P64 = host(p64)
    del p64
    g = rw_oracle.normalize(c.vol, lo, hi)
    for s in (2, 3):
        rel = c_oracle.residual(g, c.labels, s, c.beta, P64[s - 1])
        assert rel <= 1.05e-6, (s, rel)
    assert np.max(np.abs(P64.sum(0) - 1.0)) < 1e-12
    seeded = c.labels > 0
    for s in (1, 2, 3):
        assert np.all(P64[s - 1][seeded] == (c.labels[seeded] == s))

def test_sphere128_gradients_vs_central_differences(rw):
    """128^3 sphere, sigma 0.1, 500 seeds per label, beta 120, loss
    sum (x_fg - mask)^2: adjoint dL/dbeta (h 1e-4) and dL/dg on 64 sampled
    voxels (h 1e-3; 32 near the sphere surface, 32 uniform) against central
    differences of float64 solves at tol 1e-12 from x0 = 0."""
    from oracle import rw_oracle
    c = sphere_case(n=128, radius=40, sigma=0.1, seed_radius=20, corner=16, n_seeds=500,
                    beta=120.0, seed=4)
    lo, hi = c.norm_range()
    g = rw_oracle.normalize(c.vol, lo, hi)
    gd, lab, md = dev(g), dev(c.labels), dev(c.truth.astype(np.float64))

    def loss(gg, b):
        prob, _ = rw.solve(gg, lab, 2, b, tol=1e-12, precision="fp64", lo=0.0, hi=1.0, argmax=False)
        return float(((prob[1] - md) ** 2).sum())

    prob, _ = rw.solve(gd, lab, 2, 120.0, tol=1e-12, precision="fp64", lo=0.0, hi=1.0)
    dg, db = rw.solve_backward(gd, lab, 2, 120.0, 2, prob[1], 2 * (prob[1] - md), tol=1e-12)
    h = 1e-4
    fd_b = (loss(gd, 120.0 + h) - loss(gd, 120.0 - h)) / (2 * h)
    assert abs(fd_b - db) <= 1e-4 * abs(fd_b), (fd_b, db)
    rng = np.random.default_rng(4)
    dist = np.sqrt(((np.indices(g.shape) - 63.5) ** 2).sum(0)).ravel()
    unk = c.labels.ravel() == 0
    near = np.flatnonzero((np.abs(dist - 40) <= 2) & unk)
    pick = np.concatenate([rng.choice(near, 32, replace=False),
                           rng.choice(np.flatnonzero(unk), 32, replace=False)])
    hg = 1e-3
    fds, ads = [], []
    for v in pick:
        gp = gd.clone().view(-1)
        gm = gd.clone().view(-1)
        gp[v] += hg
        gm[v] -= hg
        fds.append((loss(gp.view(g.shape), 120.0) - loss(gm.view(g.shape), 120.0)) / (2 * hg))
        ads.append(float(dg.view(-1)[v]))
    fds, ads = np.array(fds), np.array(ads)
    rms = np.sqrt(np.mean(fds ** 2))
    err = np.abs(ads - fds) / np.maximum(np.abs(fds), rms)
    assert np.max(err) <= 1e-3, (np.max(err), fds[np.argmax(err)], ads[np.argmax(err)])
