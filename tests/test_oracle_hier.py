"""Pins of the oracle's coarse-to-fine pieces (hierarchical random walker,
the paper's Sec. IV-B benchmark; LOD pyramids of Sec. III-D; brick tiling of
Sec. II's chunk mapping)."""
import numpy as np
import pytest

from oracle import rw_oracle as O
from synth import blob_case, random_case


def test_downsample_mean_constant_linear_and_odd():
    a = np.full((5, 6, 7), 3.25)
    assert np.allclose(O.downsample_mean(a), 3.25)
    z, y, x = np.meshgrid(np.arange(8), np.arange(6), np.arange(4), indexing="ij")
    lin = 2.0 * x + 3.0 * y - z
    d = O.downsample_mean(lin)
    zc, yc, xc = np.meshgrid(np.arange(4), np.arange(3), np.arange(2), indexing="ij")
    assert np.allclose(d, 2.0 * (2 * xc + 0.5) + 3.0 * (2 * yc + 0.5) - (2 * zc + 0.5))
    # odd far edge: the last box averages only the voxels that exist
    b = np.arange(3, dtype=float).reshape(1, 1, 3)
    assert np.allclose(O.downsample_mean(b), [[[0.5, 2.0]]])


def test_coarse_seed_conflict_rule():
    lab = np.zeros((2, 2, 6), dtype=np.uint8)
    lab[0, 0, 0] = 2                  # block 0: only label 2
    lab[1, 1, 2] = 1
    lab[0, 1, 3] = 3                  # block 1: labels 1 and 3 -> conflict
    lab[0, 0, 4] = 3
    lab[1, 0, 5] = 3                  # block 2: two seeds of label 3
    c = O.coarse_seeds(lab)
    assert c.shape == (1, 1, 3)
    assert c.ravel().tolist() == [2, 0, 3]


def test_upsample_linear_field_exact_and_partition_of_unity():
    f = 4
    nc = (6, 5, 7)
    zc, yc, xc = np.meshgrid(*[np.arange(n, dtype=float) for n in nc], indexing="ij")
    lin = 0.5 + 0.1 * xc - 0.2 * yc + 0.05 * zc
    fine_shape = tuple(n * f for n in nc)
    up = O.upsample_trilinear(lin, fine_shape, f)
    u = [O.upsample_coords(fine_shape[k], nc[k], f) for k in range(3)]
    Z, Y, X = np.meshgrid(*u, indexing="ij")
    assert np.allclose(up, 0.5 + 0.1 * X - 0.2 * Y + 0.05 * Z, atol=1e-14)
    # interior (no clamping): u = (i + 0.5)/f - 0.5 exactly
    i = np.arange(f, fine_shape[2] - f)
    assert np.allclose(u[2][i], (i + 0.5) / f - 0.5)
    # partition of unity: probabilities summing to 1 stay summing to 1
    rng = np.random.default_rng(0)
    p = rng.random((3,) + nc)
    p /= p.sum(0)
    s = sum(O.upsample_trilinear(p[k], fine_shape, f) for k in range(3))
    assert np.allclose(s, 1.0, atol=1e-14)


def test_upsample_region_matches_full():
    coarse = np.random.default_rng(1).random((4, 5, 6))
    full = O.upsample_trilinear(coarse, (16, 20, 24), 4)
    box = O.upsample_trilinear(coarse, (16, 20, 24), 4, ((-1, 3, 5), (6, 7, 8)))
    assert np.all(np.isnan(box[0]))
    assert np.allclose(box[1:], full[0:5, 3:10, 5:13])


def test_brick_grid_offsets_give_clipped_bricks():
    bricks = O.brick_grid((1024, 1024, 1024), (64, 64, 64), (48, 20, 40))
    assert len(bricks) == 17 ** 3
    zs = sorted({s[0] for _, s in bricks})
    ys = sorted({s[1] for _, s in bricks})
    xs = sorted({s[2] for _, s in bricks})
    assert zs == [16, 48, 64] and ys == [20, 44, 64] and xs == [24, 40, 64]
    # bricks tile the volume exactly
    assert sum(int(np.prod(s)) for _, s in bricks) == 1024 ** 3


def test_brick_domain_decomposition_identity():
    """Shell values from the exact global solution => the brick solve
    reproduces the global solution inside the brick."""
    c = random_case((10, 11, 12), K=3, seeds_per_label=6, beta=12.0, seed=4)
    g = O.case_g(c)
    x = O.random_walker(g, c.labels, 3, 12.0, method="direct")
    origin, size = (2, 3, 1), (5, 4, 7)

    def shell_value(lab, zz, yy, xx):
        return x[lab - 1][zz, yy, xx]

    sl = tuple(slice(o, o + s) for o, s in zip(origin, size))
    x0 = np.zeros((3,) + size)
    xb, info = O.solve_brick(g, c.labels, origin, size, shell_value, x0, 12.0, tol=1e-13)
    for k in range(3):
        assert np.max(np.abs(xb[k] - x[k][sl])) < 1e-10


def test_brick_reproduces_linear_field_on_constant_image():
    g = np.full((12, 12, 12), 0.4)
    lab = np.zeros(g.shape, dtype=np.uint8)
    lab[0, 0, 0] = 1
    lab[-1, -1, -1] = 2
    lin = lambda zz, yy, xx: 0.3 + 0.02 * xx + 0.01 * yy - 0.015 * zz  # noqa: E731
    origin, size = (3, 2, 4), (6, 7, 5)

    def shell_value(lab_, zz, yy, xx):
        return lin(zz, yy, xx) if lab_ == 2 else 1 - lin(zz, yy, xx)

    xb, _ = O.solve_brick(g, lab, origin, size, shell_value, np.zeros((2,) + size), 80.0,
                          tol=1e-13, solve_labels=[1, 2])
    Z, Y, X = np.meshgrid(*[np.arange(o, o + s) for o, s in zip(origin, size)], indexing="ij")
    assert np.max(np.abs(xb[1] - lin(Z, Y, X))) < 1e-10
    assert np.max(np.abs(xb[0] - (1 - lin(Z, Y, X)))) < 1e-10


def test_classify_rules():
    shape = (8, 8, 8)
    lab = np.zeros(shape, dtype=np.uint8)
    P = np.zeros((2, 6, 6, 6))
    P[0] = 1.0                          # certain background everywhere
    assert not O.classify_brick(P, lab, shape, (1, 1, 1), (4, 4, 4))
    P2 = P.copy()
    P2[:, 0, 2, 2] = [0.5, 0.5]         # uncertain value on the face shell
    assert O.classify_brick(P2, lab, shape, (1, 1, 1), (4, 4, 4))
    P3 = P.copy()
    P3[:, 0, 0, 0] = [0.5, 0.5]         # frame corner: not a face neighbour
    assert not O.classify_brick(P3, lab, shape, (1, 1, 1), (4, 4, 4))
    lab2 = lab.copy()
    lab2[2, 2, 2] = 2                   # seed contradicting the argmax
    assert O.classify_brick(P, lab2, shape, (1, 1, 1), (4, 4, 4))
    P4 = P.copy()
    P4[:, 2, 2, 2] = [0.98, 0.02]       # thresholds are strict
    assert not O.classify_brick(P4, lab, shape, (1, 1, 1), (4, 4, 4))


def test_hierarchical_pipeline_small():
    c = blob_case(shape=(32, 32, 32), n_blobs=3, K=3, seeds_per_label=30, sigma=0.05,
                  rmin=4, rmax=8, seed=7, dtype="u16")
    g = O.case_g(c)
    res = O.hierarchical_rw(g, c.labels, 3, 150.0, levels=2, brick=(8, 8, 8), offset=(0, 4, 2))
    prob = res["prob"]
    seeded = c.labels > 0
    for s in range(1, 4):
        assert np.all(prob[s - 1][seeded] == (c.labels[seeded] == s))
    assert np.max(np.abs(prob.sum(0) - 1.0)) < 1e-4
    assert 0 < res["active"].sum() < len(res["bricks"])
    assert prob.min() > -1e-4 and prob.max() < 1 + 1e-4
