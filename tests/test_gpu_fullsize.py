"""Parity at the full sizes of the benchmark configurations, through
properties the CPU oracle can check at any size: its own float64 residual of
the GPU's solutions, mixed vs float64 agreement, partition of unity, exact
seeds; and finite differences of the 128^3 differentiable case."""
import numpy as np
import pytest

from synth import blob_case, sphere_case
from tests._helpers import assert_parity, dev, host, progress

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
    import torch
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
    grad_prob = torch.stack([torch.zeros_like(md), 2 * (prob[1] - md)])
    dg, db = rw.solve_backward(gd, lab, 2, 120.0, prob, grad_prob, tol=1e-12)
    db = float(db)
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


@pytest.mark.timeout(900)
def test_hier1024_sampled_bricks_vs_oracle(rw, request):
    """The full-size hierarchical workload (1024^3 uint16, 64 blobs, 8000
    seeds per label, K = 3, 64^3 bricks on the offset grid, the bench's tile
    shapes): six of the GPU's active bricks (lowest and highest GPU iteration
    counts, two clipped border bricks, two others) equal the oracle's solves
    of those bricks, which start from the oracle's own float64 levels and its
    own float64 coarse solution (labels 2 and 3; label 1 as their
    complement), brick solves by the C oracle.  Both sides stop at relative
    residual 1e-8, so the comparison is not limited by the stopping rule."""
    import time

    import torch
    from oracle import c_oracle, rw_oracle as O
    t0 = time.perf_counter()

    def say(msg):  # progress on the terminal: the oracle's part is long
        progress(request, f"hier1024 oracle test, {time.perf_counter() - t0:.0f} s: {msg}")
    tol = 1e-8
    say("generating the 1024^3 volume")
    c = blob_case(shape=(1024, 1024, 1024), n_blobs=64, K=3, seeds_per_label=8000, sigma=0.08,
                  bg=0.2, rmin=10.0, rmax=60.0, beta=150.0, seed=3, dtype="u16")
    say("volume generated; GPU hierarchical solve")
    brick, offset = (64, 64, 64), (48, 20, 40)
    prob, info = rw.hierarchical_solve(dev(c.vol), dev(c.labels), 3, c.beta, levels=2,
                                       brick=brick, offset=offset, tol=tol,
                                       coarse_precision="mixed", brick_precision="mixed",
                                       level_dtype=torch.float32, return_info=True)
    act = [b for b, a in zip(info["bricks"], info["active"]) if a]
    its = [max(i) for i in info["brick_iters"]]
    say(f"GPU done: {len(act)} active bricks, iterations {min(its)}..{max(its)}")
    assert len(act) == len(its) > 1000
    order = np.argsort(its)
    clipped = [i for i, (o, s) in enumerate(act) if min(s) < 64]
    rng = np.random.default_rng(7)
    pick = [int(order[0]), int(order[-1]), clipped[0], clipped[-1]]
    pick += [int(i) for i in rng.choice(len(act), 2, replace=False)]
    gpu = {}
    for i in pick:
        o, s = act[i]
        gpu[i] = host(prob[:, o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]])
    del prob
    torch.cuda.empty_cache()
    # the oracle's own levels and coarse solution (float64)
    say("oracle levels")
    g = O.case_g(c)
    g2, l2 = O.downsample_mean(O.downsample_mean(g)), O.coarse_seeds(O.coarse_seeds(c.labels))
    coarse = []
    for lab in (2, 3):
        say(f"oracle coarse solve of label {lab}")
        coarse.append(c_oracle.solve_box(g2, l2, lab, c.beta, tol=tol)[0])
    coarse = np.stack(coarse)
    for i in pick:
        o, s = (tuple(v) for v in act[i])
        say(f"oracle brick {o} {s}")
        # upsampled coarse values over the brick and its one-voxel frame
        # (frame voxels outside the volume are ignored by the solve)
        frame = np.stack([O.upsample_trilinear(coarse[k], c.shape, 4,
                                               (tuple(a - 1 for a in o), tuple(b + 2 for b in s)))
                          for k in range(2)])
        xb = np.stack([c_oracle.solve_box(g, c.labels, lab, c.beta, tol=tol, box=(o, s),
                                          shell=frame[k], x0=frame[k][1:-1, 1:-1, 1:-1])[0]
                       for k, lab in enumerate((2, 3))])
        ref = np.concatenate([1.0 - xb.sum(0, keepdims=True), xb])
        assert_parity(gpu[i], ref, what=f"brick {o} {s} ({its[i]} GPU iterations)")
