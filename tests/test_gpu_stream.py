"""Streamed (out-of-core-shaped) hierarchical solve: bricks through a device
pool must give exactly the resident pipeline's result, and the pool-mode
brick solve must match the oracle brick by brick."""
import numpy as np
import pytest

from synth import blob_case
from tests._helpers import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    from paper_2509_26213_amd import rw as m
    m.lib()
    return m


def test_streamed_equals_resident(rw):
    import torch
    from paper_2509_26213_amd.stream import streamed_solve
    c = blob_case(shape=(64, 96, 80), n_blobs=8, K=4, seeds_per_label=40, sigma=0.06, rmin=5,
                  rmax=14, seed=41, dtype="u16")
    prob_s, info = streamed_solve(c.vol, c.labels, 4, c.beta, brick=(32, 32, 32), pool=3,
                                  tol=1e-6, levels=2, precision="mixed")
    prob_r, rinfo = rw.hierarchical_solve(dev(c.vol), dev(c.labels), 4, c.beta, levels=2,
                                          brick=(32, 32, 32), offset=(0, 0, 0), tol=1e-6,
                                          coarse_precision="mixed", brick_precision="mixed",
                                          level_dtype=torch.float32, return_info=True)
    assert info["active_bricks"] == sum(rinfo["active"]) > 3
    assert info["bricks"] == len(rinfo["bricks"])
    assert np.array_equal(prob_s, host(prob_r))
    assert info["h2d_bytes"] > c.vol.nbytes


def test_streamed_float32_normalises_like_resident(rw):
    """A float32 volume streamed without an explicit range is min-max
    normalised over the whole volume, as the resident pipeline does: the two
    give bitwise the same probabilities."""
    import torch
    from paper_2509_26213_amd.stream import streamed_solve
    c = blob_case(shape=(48, 64, 70), n_blobs=6, K=3, seeds_per_label=30, sigma=0.06, rmin=5,
                  rmax=12, seed=45, dtype="f32")
    prob_s, info = streamed_solve(c.vol, c.labels, 3, c.beta, brick=(32, 32, 32), pool=2,
                                  tol=1e-6, levels=2, precision="mixed")
    prob_r = rw.hierarchical_solve(dev(c.vol), dev(c.labels), 3, c.beta, levels=2,
                                   brick=(32, 32, 32), offset=(0, 0, 0), tol=1e-6,
                                   coarse_precision="mixed", brick_precision="mixed",
                                   level_dtype=torch.float32)
    assert info["active_bricks"] >= 2
    assert np.array_equal(prob_s, host(prob_r))


def test_streamed_labels_only(rw):
    """Labels-only output (device argmax, uint8 over PCIe) equals the argmax
    of the streamed probabilities, lowest label on ties."""
    from paper_2509_26213_amd.stream import streamed_solve
    c = blob_case(shape=(40, 70, 66), n_blobs=6, K=3, seeds_per_label=30, sigma=0.06, rmin=5,
                  rmax=12, seed=43, dtype="u16")
    prob, _ = streamed_solve(c.vol, c.labels, 3, c.beta, brick=(16, 32, 32), pool=4,
                             tol=1e-6, levels=2, precision="mixed")
    lab = np.zeros(c.shape, np.uint8)
    lab_s, info = streamed_solve(c.vol, c.labels, 3, c.beta, brick=(16, 32, 32), pool=4,
                                 tol=1e-6, levels=2, precision="mixed", labels_out=lab)
    assert lab_s is lab
    assert np.array_equal(lab, (np.argmax(prob, axis=0) + 1).astype(np.uint8))
    seeded = c.labels > 0
    assert np.array_equal(lab[seeded], c.labels[seeded])


def test_argmax_ties_and_dtypes(rw):
    import torch
    rng = np.random.default_rng(5)
    for dt in (torch.float32, torch.float64):
        p = rng.integers(0, 3, size=(4, 1000)).astype(np.float64)  # many ties
        am = host(rw.argmax(torch.tensor(p, dtype=dt, device="cuda")))
        assert np.array_equal(am, (np.argmax(p, axis=0) + 1).astype(np.uint8))


@pytest.mark.parametrize("pad", [0, 1 << 29])
def test_pool_bricks_match_resident_bricks(rw, pad):
    """A brick solved inside its own halo sub-volume equals the same brick
    solved inside the full volume (bitwise); with pad, the pool holds more
    voxels than one plane of a volume may (2^29), which a pool may."""
    import torch
    c = blob_case(shape=(40, 48, 56), n_blobs=5, K=3, seeds_per_label=30, sigma=0.06, rmin=4,
                  rmax=12, seed=7, dtype="u16")
    vol, lab = dev(c.vol), dev(c.labels)
    g1, l1 = rw.downsample(vol, lab, out_dtype=torch.float64)
    g2, l2 = rw.downsample(g1, l1, lo=0.0, hi=1.0, out_dtype=torch.float64)
    coarse, _ = rw.solve(g2, l2, 3, c.beta, tol=1e-10, precision="fp64", lo=0.0, hi=1.0)
    bricks = [((0, 0, 0), (16, 16, 16)), ((8, 16, 24), (16, 20, 18)), ((24, 32, 40), (16, 16, 16))]
    ref, _ = rw.solve_bricks(vol, lab, 3, c.beta, coarse, 4, bricks, precision="mixed")
    R = host(ref)
    # pool: each brick with its clipped one-voxel halo
    subs, local, chunks_v, chunks_l = [], [], [], []
    off = 0
    for o, s in bricks:
        lo = [max(o[a] - 1, 0) for a in range(3)]
        hi = [min(o[a] + s[a] + 1, c.shape[a]) for a in range(3)]
        sv = c.vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        subs.append((off, sv.shape, tuple(lo)))
        local.append((tuple(o[a] - lo[a] for a in range(3)), s))
        chunks_v.append(sv.ravel())
        chunks_l.append(c.labels[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].ravel())
        off += sv.size
    hv = np.zeros(off + pad, np.uint16)
    hl = np.zeros(off + pad, np.uint8)
    hv[:off] = np.concatenate(chunks_v)
    hl[:off] = np.concatenate(chunks_l)
    pv, pl = dev(hv.reshape(1, 1, -1)), dev(hl.reshape(1, 1, -1))
    del hv, hl
    pp, _ = rw.solve_bricks(pv, pl, 3, c.beta, coarse, 4, local, subvols=subs, precision="mixed",
                            lo=0.0, hi=65535.0)
    P = host(pp.reshape(3, -1)[:, :off])
    for (off, dims, lo), (ob, s), (o, _) in zip(subs, local, bricks):
        blk = P[:, off:off + int(np.prod(dims))].reshape((3,) + tuple(dims))
        inner = blk[:, ob[0]:ob[0] + s[0], ob[1]:ob[1] + s[1], ob[2]:ob[2] + s[2]]
        want = R[:, o[0]:o[0] + s[0], o[1]:o[1] + s[1], o[2]:o[2] + s[2]]
        assert np.array_equal(inner, want)
