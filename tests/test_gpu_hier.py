"""GPU parity of the coarse-to-fine pieces against the oracle: LOD step,
coarse seeds, brick classification, upsampled fill, batched brick solves and
the whole hierarchical pipeline."""
import numpy as np
import pytest

from oracle import rw_oracle as O
from synth import blob_case
from tests._helpers import assert_parity, dev, host, near_threshold

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    from paper_2509_26213_amd import rw as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def case():
    # ragged sizes (not multiples of the brick or of 4), three labels, u16
    return blob_case(shape=(45, 52, 70), n_blobs=6, K=3, seeds_per_label=40, sigma=0.06,
                     rmin=5, rmax=14, seed=31, dtype="u16")


@pytest.fixture(scope="module")
def coarse_ref(case):
    """Oracle levels and coarse solution (float64), the GPU brick stage's input."""
    g = O.case_g(case)
    g1, l1 = O.downsample_mean(g), O.coarse_seeds(case.labels)
    g2, l2 = O.downsample_mean(g1), O.coarse_seeds(l1)
    coarse = O.random_walker(g2, l2, case.K, case.beta, method="pcg", tol=1e-10)
    return g, (g1, l1), (g2, l2), coarse


def test_downsample_matches_oracle(rw, case, coarse_ref):
    import torch
    g, (g1, l1), (g2, l2), _ = coarse_ref
    vol, lab = dev(case.vol), dev(case.labels)
    d1, dl1 = rw.downsample(vol, lab, out_dtype=torch.float64)
    d2, dl2 = rw.downsample(d1, dl1, lo=0.0, hi=1.0, out_dtype=torch.float64)
    assert np.allclose(host(d1), g1, rtol=0, atol=1e-15)
    assert np.allclose(host(d2), g2, rtol=0, atol=1e-15)
    assert np.array_equal(host(dl1), l1) and np.array_equal(host(dl2), l2)
    f32, _ = rw.downsample(vol, None, out_dtype=torch.float32)
    assert np.allclose(host(f32), g1, rtol=1e-6, atol=1e-7)


def _up(coarse, shape, f, origin, size):
    return np.stack([O.upsample_trilinear(coarse[k], shape, f, (origin, size))
                     for k in range(coarse.shape[0])])


@pytest.mark.parametrize("offset", [(0, 0, 0), (5, 3, 7)])
def test_classify_matches_oracle(rw, case, coarse_ref, offset):
    _, _, _, coarse = coarse_ref
    brick = (16, 16, 16)
    cands, active = rw.classify_bricks(dev(coarse), dev(case.labels), 4, brick, offset)
    ref = O.brick_grid(case.shape, brick, offset)
    assert [tuple(map(tuple, b)) for b in cands] == [(tuple(o), tuple(s)) for o, s in ref]
    for (o, s), a in zip(ref, active):
        P = _up(coarse, case.shape, 4, tuple(np.array(o) - 1), tuple(np.array(s) + 2))
        assert O.classify_brick(P, case.labels, case.shape, o, s) == a, (o, s)
    assert 0 < sum(active) < len(active)


def test_fill_matches_upsampling(rw, case, coarse_ref):
    import torch
    _, _, _, coarse = coarse_ref
    bricks = O.brick_grid(case.shape, (16, 16, 16), (0, 0, 0))[::3]
    prob = torch.full((3,) + case.shape, -1.0, dtype=torch.float32, device="cuda")
    rw.fill_bricks(dev(coarse), dev(case.labels), 4, bricks, prob)
    P = host(prob)
    for o, s in bricks:
        sl = tuple(slice(a, a + b) for a, b in zip(o, s))
        ref = _up(coarse, case.shape, 4, o, s)
        lab = case.labels[sl]
        for k in range(3):
            r = ref[k].copy()
            r[lab > 0] = (lab[lab > 0] == k + 1)
            assert np.allclose(P[k][sl], r, atol=1e-6)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_brick_solves_match_oracle(rw, case, coarse_ref, precision):
    g, _, _, coarse = coarse_ref
    offset = (5, 3, 7)
    cands, active = rw.classify_bricks(dev(coarse), dev(case.labels), 4, (16, 16, 16), offset)
    act = [b for b, a in zip(cands, active) if a][:12]
    prob, iters, st = rw.solve_bricks(dev(case.vol), dev(case.labels), 3, case.beta, dev(coarse), 4,
                                      act, tol=1e-6, precision=precision, return_stats=True)
    P = host(prob)
    assert st["status"] == 0
    for (o, s), it in zip(act, iters):
        o, s = tuple(o), tuple(s)
        Pf = _up(coarse, case.shape, 4, tuple(np.array(o) - 1), tuple(np.array(s) + 2))

        def shell_value(lab, zz, yy, xx, Pf=Pf, o=o):
            return Pf[lab - 1][zz - o[0] + 1, yy - o[1] + 1, xx - o[2] + 1]

        x0 = Pf[:, 1:-1, 1:-1, 1:-1]
        xb, info = O.solve_brick(g, case.labels, o, s, shell_value, x0, case.beta, tol=1e-6)
        sl = tuple(slice(a, a + b) for a, b in zip(o, s))
        assert_parity(P[:, sl[0], sl[1], sl[2]], xb, what=f"brick {o} {precision}")
        if precision == "fp64":
            # same algorithm, same x0, same stopping rule: the same count +- 1
            for r in range(2):
                assert abs(it[r] - info[r + 1]["iters"]) <= 1, (it, info)


@pytest.mark.parametrize("vx", [1, 2])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_deep_brick_tiles_match_oracle(rw, case, coarse_ref, monkeypatch, precision, vx):
    """Bricks 40 and 45 planes deep on 64-plane tiles: the residual's cache of
    interpolated x-halo shell values is refilled within a tile (every 32
    planes), and the solves still meet the oracle's (float64: the same
    iteration counts to within one)."""
    g, _, _, coarse = coarse_ref
    monkeypatch.setenv("RW_BRICK_BY", "8")
    monkeypatch.setenv("RW_BRICK_VX", str(vx))
    monkeypatch.setenv("RW_BRICK_ZC", "64")
    cands, active = rw.classify_bricks(dev(coarse), dev(case.labels), 4, (48, 48, 48), (5, 3, 7))
    act = [b for b, a in zip(cands, active) if a and b[1][0] > 32][:4]
    assert act
    prob, iters, st = rw.solve_bricks(dev(case.vol), dev(case.labels), 3, case.beta, dev(coarse), 4,
                                      act, tol=1e-8, precision=precision, return_stats=True)
    assert st["status"] == 0 and st["tile"]["zc"] == 64
    P = host(prob)
    for (o, s), it in zip(act, iters):
        o, s = tuple(o), tuple(s)
        Pf = _up(coarse, case.shape, 4, tuple(np.array(o) - 1), tuple(np.array(s) + 2))

        def shell_value(lab, zz, yy, xx, Pf=Pf, o=o):
            return Pf[lab - 1][zz - o[0] + 1, yy - o[1] + 1, xx - o[2] + 1]

        xb, info = O.solve_brick(g, case.labels, o, s, shell_value, Pf[:, 1:-1, 1:-1, 1:-1],
                                 case.beta, tol=1e-8)
        sl = tuple(slice(a, a + b) for a, b in zip(o, s))
        assert_parity(P[:, sl[0], sl[1], sl[2]], xb, what=f"deep brick {o} {s} {precision}")
        if precision == "fp64":
            for r in range(2):
                assert abs(it[r] - info[r + 1]["iters"]) <= 1, (it, info)


@pytest.mark.parametrize("by,zc,xcd,vx", [(4, 16, 0, 1), (8, 64, 0, 1), (16, 8, 1, 1),
                                          (8, 5, 1, 1), (4, 64, 0, 2), (8, 6, 1, 2)])
def test_brick_tile_shapes_match_oracle(rw, case, coarse_ref, monkeypatch, by, zc, xcd, vx):
    """Every brick tile shape (waves per block, rows per lane, planes per
    tile, worklist order) gives the oracle's brick solutions: ragged 32^3
    bricks clipped by the volume border, float64."""
    g, _, _, coarse = coarse_ref
    monkeypatch.setenv("RW_BRICK_BY", str(by))
    monkeypatch.setenv("RW_BRICK_VX", str(vx))
    monkeypatch.setenv("RW_BRICK_ZC", str(zc))
    monkeypatch.setenv("RW_BRICK_XCD", str(xcd))
    cands, active = rw.classify_bricks(dev(coarse), dev(case.labels), 4, (32, 32, 32), (5, 3, 7))
    act = [b for b, a in zip(cands, active) if a][:6]
    prob, iters, st = rw.solve_bricks(dev(case.vol), dev(case.labels), 3, case.beta, dev(coarse), 4,
                                      act, tol=1e-6, precision="fp64", return_stats=True)
    assert st["status"] == 0 and st["tile"]["by"] == by and st["tile"]["vx"] == vx
    P = host(prob)
    for (o, s), it in zip(act, iters):
        o, s = tuple(o), tuple(s)
        Pf = _up(coarse, case.shape, 4, tuple(np.array(o) - 1), tuple(np.array(s) + 2))

        def shell_value(lab, zz, yy, xx, Pf=Pf, o=o):
            return Pf[lab - 1][zz - o[0] + 1, yy - o[1] + 1, xx - o[2] + 1]

        xb, info = O.solve_brick(g, case.labels, o, s, shell_value, Pf[:, 1:-1, 1:-1, 1:-1],
                                 case.beta, tol=1e-6)
        sl = tuple(slice(a, a + b) for a, b in zip(o, s))
        assert_parity(P[:, sl[0], sl[1], sl[2]], xb, what=f"brick {o} tile {by}x{zc}")
        for r in range(2):
            assert abs(it[r] - info[r + 1]["iters"]) <= 1, (it, info)


def test_bricks_untouched_outside(rw, case, coarse_ref):
    import torch
    _, _, _, coarse = coarse_ref
    b = [((0, 0, 0), (16, 20, 24))]
    prob = torch.full((3,) + case.shape, 7.0, dtype=torch.float32, device="cuda")
    rw.solve_bricks(dev(case.vol), dev(case.labels), 3, case.beta, dev(coarse), 4, b,
                    prob_out=prob, precision="mixed")
    P = host(prob)
    inside = np.zeros(case.shape, bool)
    inside[:16, :20, :24] = True
    assert np.all(P[:, ~inside] == 7.0)
    assert np.all(P[:, inside] != 7.0)


def test_hierarchical_coarse_tolerance_induced_gap(rw, case, coarse_ref):
    """At tol 1e-6 this coarse grid is ill-conditioned enough that a
    tolerance-stopped solve is 3e-3 away from the exact solution, so the
    complement background differs from an independent background solve by
    that much.  The solved labels (2, 3) follow the oracle's PCG run."""
    import torch
    g, _, (g2, l2), _ = coarse_ref
    xs = O.random_walker(g2, l2, 3, case.beta, method="pcg", tol=1e-6)
    xe = O.random_walker(g2, l2, 3, case.beta, method="direct")
    assert np.max(np.abs(xs - xe)) > 1e-5          # the disclosed gap
    prob, _ = rw.solve(dev(g2), dev(l2), 3, case.beta, tol=1e-6, precision="fp64", lo=0.0, hi=1.0)
    assert np.max(np.abs(host(prob)[1:] - xs[1:])) < 1e-5


HIER_GRID = dict(levels=2, brick=(16, 16, 16), offset=(5, 3, 7))


@pytest.fixture(scope="module")
def hier_ref(case):
    """The oracle's own hierarchical solve of `case` at tol 1e-9 (the second
    parity run for the tolerance-induced gap): its levels, coarse solve,
    brick list and brick solves."""
    return O.hierarchical_rw(O.case_g(case), case.labels, 3, case.beta, tol=1e-9, **HIER_GRID)


def _agree_with_oracle(P, ref, labels, gpu_active=None, skip=(), what=""):
    """Bricks whose activity differs from the oracle's must be within 1e-4
    of a decision; every other brick (not in skip) meets the parity bar."""
    n_diff = 0
    for i, ((o, s), a) in enumerate(zip(ref["bricks"], ref["active"])):
        if gpu_active is not None and gpu_active[i] != a:
            assert near_threshold(ref["coarse"], labels, 4, o, s), (what, i, o, s)
            n_diff += 1
            continue
        if i in skip:
            continue
        sl = tuple(slice(x, x + y) for x, y in zip(o, s))
        assert_parity(P[:, sl[0], sl[1], sl[2]], ref["prob"][:, sl[0], sl[1], sl[2]],
                      what=f"{what} brick {o}")
    return n_diff


@pytest.mark.parametrize("brick_precision", ["mixed", "fp64"])
def test_hierarchical_pipeline_matches_oracle(rw, case, hier_ref, brick_precision):
    """End to end at tol 1e-9 (the second parity run for a tolerance-induced
    gap): the oracle runs its own levels, coarse solve and brick list; brick
    lists agree except for bricks within 1e-4 of a threshold (checked on the
    oracle's upsampled coarse solution), probabilities agree to 1e-5 on the
    agreeing bricks."""
    brick, offset = HIER_GRID["brick"], HIER_GRID["offset"]
    ref = hier_ref
    prob, info = rw.hierarchical_solve(dev(case.vol), dev(case.labels), 3, case.beta, levels=2,
                                       brick=brick, offset=offset, tol=1e-9,
                                       coarse_precision="fp64", brick_precision=brick_precision,
                                       return_info=True)
    P = host(prob)
    assert np.max(np.abs(host(info["coarse"]) - ref["coarse"])) < 1e-5
    assert sum(ref["active"]) >= 5
    _agree_with_oracle(P, ref, case.labels, info["active"], what=brick_precision)


def test_brick_autotuner_records_a_tile_and_solves_agree(rw, case, coarse_ref):
    """rw_autotune_bricks times every candidate brick tile shape on a batch and
    records the fastest; later mixed brick solves with the same label count
    and brick size class use it and still give the oracle's brick solutions
    (ragged 32^3 bricks clipped by the volume border)."""
    g, _, _, coarse = coarse_ref
    cands, active = rw.classify_bricks(dev(coarse), dev(case.labels), 4, (32, 32, 32), (5, 3, 7))
    act = [b for b, a in zip(cands, active) if a][:6]
    vol, lab, cp = dev(case.vol), dev(case.labels), dev(coarse)
    by, rpl, zc, xcd = rw.autotune_bricks(vol, lab, 3, case.beta, cp, 4, act, precision="mixed")
    assert (by, rpl) in {(8, 2), (4, 2), (16, 1), (8, 1), (4, 1)}
    assert zc in (16, 32, 64) and xcd in (0, 1)
    prob, iters, st = rw.solve_bricks(vol, lab, 3, case.beta, cp, 4, act, tol=1e-6,
                                      precision="mixed", return_stats=True)
    assert st["status"] == 0
    t = st["tile"]
    assert (t["by"], t["vx"], t["zc"], t["xcd"]) == (by, rpl, zc, xcd)
    P = host(prob)
    for o, s in act:
        o, s = tuple(o), tuple(s)
        Pf = _up(coarse, case.shape, 4, tuple(np.array(o) - 1), tuple(np.array(s) + 2))

        def shell_value(lab_, zz, yy, xx, Pf=Pf, o=o):
            return Pf[lab_ - 1][zz - o[0] + 1, yy - o[1] + 1, xx - o[2] + 1]

        xb, _ = O.solve_brick(g, case.labels, o, s, shell_value, Pf[:, 1:-1, 1:-1, 1:-1],
                              case.beta, tol=1e-6)
        sl = tuple(slice(a, a + b) for a, b in zip(o, s))
        assert_parity(P[:, sl[0], sl[1], sl[2]], xb, what=f"brick {o} after autotune")


@pytest.mark.parametrize("roi", [((0, 20), (10, 30), (30, 70)), ((40, 45), (0, 52), (0, 9))])
def test_region_of_interest_equals_full_solve(rw, case, roi):
    """Lazy evaluation of a region: only the bricks meeting the box are solved
    or filled, and inside the box the result equals the full hierarchical
    solve bit for bit (a brick's solve does not depend on its batch)."""
    import torch
    brick, offset = (16, 16, 16), (5, 3, 7)
    vol, lab = dev(case.vol), dev(case.labels)
    full, finfo = rw.hierarchical_solve(vol, lab, 3, case.beta, levels=2, brick=brick,
                                        offset=offset, brick_precision="mixed",
                                        return_info=True)
    part, pinfo = rw.hierarchical_solve(vol, lab, 3, case.beta, levels=2, brick=brick,
                                        offset=offset, brick_precision="mixed", roi=roi,
                                        return_info=True)
    assert torch.equal(finfo["coarse"], pinfo["coarse"])
    n_eval = sum(pinfo["evaluated"])
    assert 0 < n_eval < len(pinfo["bricks"])
    sl = tuple(slice(a, b) for a, b in roi)
    assert torch.equal(part[:, sl[0], sl[1], sl[2]], full[:, sl[0], sl[1], sl[2]])
    # every voxel of an unevaluated brick is left 0
    for (o, s), e in zip(pinfo["bricks"], pinfo["evaluated"]):
        if not e:
            bs = tuple(slice(a, a + b) for a, b in zip(o, s))
            assert not bool(part[:, bs[0], bs[1], bs[2]].any())


@pytest.mark.parametrize("roi", [((0, 20), (10, 30), (30, 70)), ((40, 45), (0, 52), (0, 9))])
def test_region_of_interest_matches_oracle(rw, case, hier_ref, roi):
    """Lazy evaluation of a region at tol 1e-9 against the oracle's full
    hierarchical solve: inside the box every voxel meets the parity bar
    (bricks whose activity differs from the oracle's must be within 1e-4 of
    a decision)."""
    vol, lab = dev(case.vol), dev(case.labels)
    part, pinfo = rw.hierarchical_solve(vol, lab, 3, case.beta, tol=1e-9, coarse_precision="fp64",
                                        brick_precision="mixed", roi=roi, return_info=True,
                                        **HIER_GRID)
    P = host(part)
    ref = hier_ref
    inbox = np.zeros(case.shape, bool)
    inbox[tuple(slice(a, b) for a, b in roi)] = True
    for i, ((o, s), a) in enumerate(zip(ref["bricks"], ref["active"])):
        if not pinfo["evaluated"][i]:
            continue
        if pinfo["active"][i] != a:
            assert near_threshold(ref["coarse"], case.labels, 4, o, s), (i, o, s)
            continue
        sl = tuple(slice(x, x + y) for x, y in zip(o, s))
        m = inbox[sl]
        assert m.any()
        assert_parity(P[:, sl[0], sl[1], sl[2]][:, m], ref["prob"][:, sl[0], sl[1], sl[2]][:, m],
                      what=f"roi brick {o}")


def test_seed_edit_resolve_matches_oracle(rw, case, hier_ref):
    """A seed edit re-solved incrementally at tol 1e-9 against the oracle's
    full hierarchical solve of the edited seeds: redone bricks meet the
    parity bar, kept bricks are within change_tol (1e-4) of it, bricks whose
    activity differs are within 1e-4 of a decision."""
    kw = dict(tol=1e-9, coarse_precision="fp64", brick_precision="mixed", **HIER_GRID)
    vol, lab = dev(case.vol), dev(case.labels)
    prev, pinfo = rw.hierarchical_solve(vol, lab, 3, case.beta, return_info=True, **kw)
    new = case.labels.copy()
    blk = new[30:33, 20:23, 40:43]
    blk[blk == 0] = 3
    inc, info = rw.resolve_after_seed_edit(vol, lab, dev(new), 3, case.beta, prev, pinfo,
                                           change_tol=1e-4, **kw)
    ref = O.hierarchical_rw(O.case_g(case), new, 3, case.beta, tol=1e-9, **HIER_GRID)
    P = host(inc)
    redo = set(info["resolved"]) | set(info["refilled"])
    assert redo
    for i, ((o, s), a) in enumerate(zip(ref["bricks"], ref["active"])):
        if info["active"][i] != a:
            assert near_threshold(ref["coarse"], new, 4, o, s), (i, o, s)
            continue
        sl = tuple(slice(x, x + y) for x, y in zip(o, s))
        err = np.max(np.abs(P[:, sl[0], sl[1], sl[2]] - ref["prob"][:, sl[0], sl[1], sl[2]]))
        assert err <= (1e-5 if i in redo else 1e-4 + 1e-5), (i, i in redo, err)


def test_seed_edit_resolve_matches_full_solve(rw, case):
    """Interactive seed edit: the warm-started re-solve redoes only the bricks
    the edit reaches (holding or bordering an edited voxel, or whose coarse
    data moved by more than change_tol), keeps the others bit for bit, and
    agrees with a full re-solve to change_tol (kept bricks, maximum principle)
    and to the solver tolerance on the redone ones."""
    import torch
    brick, offset = (16, 16, 16), (5, 3, 7)
    kw = dict(levels=2, brick=brick, offset=offset, tol=1e-8, coarse_precision="fp64",
              brick_precision="mixed")
    vol, lab = dev(case.vol), dev(case.labels)
    prev, pinfo = rw.hierarchical_solve(vol, lab, 3, case.beta, return_info=True, **kw)
    new = case.labels.copy()
    blk = new[30:33, 20:23, 40:43]
    blk[blk == 0] = 3
    assert (new != case.labels).sum() > 0
    newd = dev(new)
    full, _ = rw.hierarchical_solve(vol, newd, 3, case.beta, return_info=True, **kw)
    inc, info = rw.resolve_after_seed_edit(vol, lab, newd, 3, case.beta, prev, pinfo,
                                           change_tol=1e-4, **kw)
    assert len(info["resolved"]) >= 1
    redo = set(info["resolved"]) | set(info["refilled"])
    P, F, Q = host(inc), host(full), host(prev)
    for i, (o, s) in enumerate(info["bricks"]):
        sl = tuple(slice(a, a + b) for a, b in zip(o, s))
        a, f, q = P[:, sl[0], sl[1], sl[2]], F[:, sl[0], sl[1], sl[2]], Q[:, sl[0], sl[1], sl[2]]
        if i in redo:
            assert np.max(np.abs(a - f)) <= 1e-5, (i, np.max(np.abs(a - f)))
        else:
            assert np.array_equal(a, q), i
            assert np.max(np.abs(a - f)) <= 1e-4 + 1e-5, (i, np.max(np.abs(a - f)))
    seeded = new > 0
    for s_ in (1, 2, 3):
        assert np.all(P[s_ - 1][seeded] == (new[seeded] == s_))


@pytest.mark.parametrize("K", [3, 4])
def test_persistent_brick_kernel_matches_oracle(rw, case, coarse_ref, monkeypatch, K):
    """The persistent form of the batched brick solve (one launch: each
    block claims bricks from an atomic queue and runs a brick's whole CG in
    block-local state), on the default tiles of two and three solved labels:
    ragged 16^3 and 32^3 bricks against the oracle's brick solves."""
    monkeypatch.setenv("RW_BRICK_PERSIST", "1")
    if K == 3:
        c, g, coarse = case, coarse_ref[0], coarse_ref[3]
    else:
        c = blob_case(shape=(45, 70, 90), n_blobs=8, K=4, seeds_per_label=40, sigma=0.06, rmin=5,
                      rmax=14, seed=53, dtype="u16")
        g = O.case_g(c)
        g2, l2 = O.downsample_mean(O.downsample_mean(g)), O.coarse_seeds(O.coarse_seeds(c.labels))
        coarse = O.random_walker(g2, l2, 4, c.beta, method="pcg", tol=1e-10)
    for size in ((16, 16, 16), (32, 32, 32)):
        cands, active = rw.classify_bricks(dev(coarse), dev(c.labels), 4, size, (5, 3, 7))
        act = [b for b, a in zip(cands, active) if a][:24]
        prob, iters, st = rw.solve_bricks(dev(c.vol), dev(c.labels), K, c.beta, dev(coarse), 4,
                                          act, tol=1e-6, precision="mixed", return_stats=True)
        assert st["status"] == 0 and st["brick_blocks"] > 0, st
        P = host(prob)
        for (o, s), it in zip(act, iters):
            o, s = tuple(o), tuple(s)
            Pf = np.stack([O.upsample_trilinear(coarse[k], c.shape, 4,
                                                (tuple(np.array(o) - 1), tuple(np.array(s) + 2)))
                           for k in range(K)])

            def shell_value(lab_, zz, yy, xx, Pf=Pf, o=o):
                return Pf[lab_ - 1][zz - o[0] + 1, yy - o[1] + 1, xx - o[2] + 1]

            xb, _ = O.solve_brick(g, c.labels, o, s, shell_value, Pf[1:, 1:-1, 1:-1, 1:-1], c.beta,
                                  tol=1e-6, solve_labels=list(range(2, K + 1)))
            sl = tuple(slice(a, a + b) for a, b in zip(o, s))
            err = np.max(np.abs(P[1:, sl[0], sl[1], sl[2]] - xb))
            assert err <= 1e-5, (o, s, err, it)


@pytest.mark.parametrize("offset", [(0, 0, 0), (5, 3, 7)])
def test_classify_with_seed_list_equals_dense_map(rw, case, coarse_ref, offset):
    """Brick activity with the seed rule taken from a seed list (the form
    the streamed pipeline uses, the fine label map never on the device)
    equals the dense-map classification, brick for brick; a seed that
    contradicts the coarse argmax makes its brick active."""
    import torch
    _, _, _, coarse = coarse_ref
    brick = (16, 16, 16)
    cands, active = rw.classify_bricks(dev(coarse), dev(case.labels), 4, brick, offset)
    flat = np.flatnonzero(case.labels)
    sidx = torch.from_numpy(flat.astype(np.int64)).cuda()
    slab = torch.from_numpy(case.labels.reshape(-1)[flat]).cuda()
    c2, a2 = rw.classify_bricks_sparse(dev(coarse), sidx, slab, case.shape, 4, brick, offset)
    assert c2 == cands and a2 == active
    # no seeds at all: only the probability rule
    _, a0 = rw.classify_bricks_sparse(dev(coarse), sidx[:0], slab[:0], case.shape, 4, brick,
                                      offset)
    nolab = np.zeros_like(case.labels)
    _, ad = rw.classify_bricks(dev(coarse), dev(nolab), 4, brick, offset)
    assert a0 == ad
    # a seed against the argmax in an otherwise certain brick
    certain = [i for i, a in enumerate(ad) if not a]
    if certain:
        o, s = cands[certain[0]]
        P = np.stack([O.upsample_trilinear(coarse[k], case.shape, 4, (tuple(o), tuple(s)))
                      for k in range(3)])
        am = int(np.argmax(P[:, 0, 0, 0])) + 1
        idx = (o[0] * case.shape[1] + o[1]) * case.shape[2] + o[2]
        _, a1 = rw.classify_bricks_sparse(dev(coarse), torch.tensor([idx], device="cuda"),
                                          torch.tensor([am % 3 + 1], dtype=torch.uint8,
                                                       device="cuda"), case.shape, 4, brick,
                                          offset)
        assert a1[certain[0]] and sum(a1) == sum(ad) + 1


def test_seed_edit_bricks_match_a_direct_count(rw, case, coarse_ref):
    """rw_seed_edit_bricks against a direct numpy count on the host: the
    bricks holding a changed voxel or one of its face neighbours, and the
    largest coarse change over each brick's footprint and one cell around."""
    import torch
    _, _, _, coarse = coarse_ref
    brick, offset = (16, 16, 16), (5, 3, 7)
    new = case.labels.copy()
    new[30:33, 20:23, 40:43][new[30:33, 20:23, 40:43] == 0] = 3
    new[0, 0, 0] = 2
    new[44, 51, 69] = 1
    rng = np.random.default_rng(3)
    coarse2 = coarse + 1e-3 * rng.standard_normal(coarse.shape) * (rng.random(coarse.shape) < 0.01)
    ed, mv = rw.seed_edit_bricks(dev(case.labels), dev(new), dev(coarse), dev(coarse2), 4, brick,
                                 offset)
    grid = O.brick_grid(case.shape, brick, offset)
    assert len(ed) == len(mv) == len(grid)
    changed = np.argwhere(case.labels != new)
    want = np.zeros(len(grid), bool)
    for i, (o, s) in enumerate(grid):
        o_, e_ = np.array(o), np.array(o) + np.array(s)
        for p in changed:
            outside = int(np.sum((p < o_) | (p >= e_)))       # axes on which p leaves the box
            near = bool(np.all((p >= o_ - 1) & (p <= e_)))    # within one voxel of it
            if outside == 0 or (outside == 1 and near):       # in the brick or its face shell
                want[i] = True
                break
    assert ed == list(want)
    dc = np.abs(coarse2 - coarse).max(0)
    for i, (o, s) in enumerate(grid):
        sl = tuple(slice(max(0, a // 4 - 1), min(n, -(-(a + b) // 4) + 1))
                   for a, b, n in zip(o, s, dc.shape))
        assert mv[i] == float(dc[sl].max()), i


def test_region_of_interest_keeps_the_levels_tiles_after_tuning(tmp_path):
    """With a tile-table entry for the level's 16^3 bricks, a region made
    only of clipped border bricks still runs on that entry's tiles (the
    pipeline passes the nominal brick size as the table key), so the box
    holds the full solve bit for bit; the same bricks solved without the key
    fall into a smaller size class and take the built-in tiles."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    table = tmp_path / "librw.tune"
    table.write_text("brick 1 2 12 4 16 0 1 0 0\n")
    code = """
import json, sys, torch
sys.path.insert(0, %r)
from paper_2509_26213_amd import rw
from synth import blob_case
c = blob_case(shape=(45, 52, 70), n_blobs=6, K=3, seeds_per_label=40, sigma=0.06, rmin=5,
              rmax=14, seed=31, dtype="u16")
vol = torch.from_numpy(c.vol).cuda(); lab = torch.from_numpy(c.labels).cuda()
kw = dict(levels=2, brick=(16, 16, 16), offset=(5, 3, 7), brick_precision="mixed", return_info=True)
roi = ((0, 3), (0, 52), (0, 70))
full, fi = rw.hierarchical_solve(vol, lab, 3, c.beta, **kw)
part, pi = rw.hierarchical_solve(vol, lab, 3, c.beta, roi=roi, **kw)
sl = tuple(slice(a, b) for a, b in roi)
act = [b for b, a, e in zip(pi["bricks"], pi["active"], pi["evaluated"]) if a and e]
_, _, st = rw.solve_bricks(vol, lab, 3, c.beta, pi["coarse"], 4, act, return_stats=True)
print(json.dumps(dict(equal=bool(torch.equal(part[(slice(None),) + sl], full[(slice(None),) + sl])),
                      n=len(act), biggest=max(s[0] * s[1] * s[2] for _, s in act),
                      full=fi["brick_stats"]["tile"], roi=pi["brick_stats"]["tile"],
                      unkeyed=st["tile"], tuned=[fi["brick_stats"]["tile_tuned"],
                                                 st["tile_tuned"]])))
""" % root
    r = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, RW_TUNE_FILE=str(table)),
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n"] > 0 and out["biggest"] < 4096, out
    assert out["tuned"] == [True, False], out
    assert out["full"] == out["roi"] and out["full"]["by"] == 4 and out["full"]["vx"] == 1, out
    assert out["unkeyed"] != out["full"], out
    assert out["equal"], out
