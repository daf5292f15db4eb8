"""GPU parity of the whole-volume solve (librw.so through the C ABI) against
the CPU oracle: weights, the matrix-free operator, FP64 and mixed Jacobi-PCG,
edge cases and error statuses."""
import os

import numpy as np
import pytest

from oracle import rw_oracle as O
from synth import blob_case, random_case, sphere_case
from tests._helpers import assert_parity, dev, host

ROOT_DIR = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    from paper_2509_26213_amd import rw as m
    m.lib()
    return m


def _case_tensors(c):
    return dev(c.vol), dev(c.labels)


# ---------------------------------------------------------------- weights

@pytest.mark.parametrize("dtype", ["f32", "u16"])
def test_build_weights_fp64_and_fp32(rw, dtype):
    c = blob_case(shape=(19, 33, 70), n_blobs=4, K=3, seeds_per_label=10, rmin=3, rmax=9,
                  seed=3, dtype=dtype)
    vol, lab = _case_tensors(c)
    lo, hi = c.norm_range()
    g = O.case_g(c)
    ref = O.weights_grid(g, c.beta)
    w64, dinv64 = rw.build_weights(vol, c.beta, "fp64", labels=lab, lo=lo, hi=hi)
    w64 = host(w64)
    assert np.allclose(w64, ref, rtol=1e-13, atol=1e-300)
    dref = np.where(c.labels == 0, 1.0 / O.degrees(g, c.beta), 0.0)
    assert np.allclose(host(dinv64), dref, rtol=1e-13)
    w32, _ = rw.build_weights(vol, c.beta, "mixed", lo=lo, hi=hi)
    w32 = host(w32).astype(np.float64)
    # float32: rounding of the exponent argument grows with |beta dg^2|
    arg = np.zeros_like(ref)
    arg[0][:, :, :-1] = c.beta * (g[:, :, 1:] - g[:, :, :-1]) ** 2
    arg[1][:, :-1, :] = c.beta * (g[:, 1:, :] - g[:, :-1, :]) ** 2
    arg[2][:-1] = c.beta * (g[1:] - g[:-1]) ** 2
    tolw = (4e-7 * arg + 1e-6) * ref + 1.2e-38
    edge = ref > 0
    assert np.all(np.abs(w32 - ref)[edge] <= tolw[edge])
    assert np.all(w32[~edge] == 0)


def test_minmax(rw):
    c = blob_case(shape=(20, 30, 40), n_blobs=3, K=3, seeds_per_label=5, rmin=3, rmax=8, seed=1)
    lo, hi = rw.minmax(dev(c.vol))
    assert lo == float(c.vol.min()) and hi == float(c.vol.max())


# ---------------------------------------------------------------- operator

@pytest.mark.parametrize("shape", [(9, 13, 70), (33, 5, 129)])
def test_operator_matches_assembled_laplacian(rw, shape):
    c = random_case(shape, K=2, seeds_per_label=20, beta=25.0, seed=5)
    vol, lab = _case_tensors(c)
    lo, hi = c.norm_range()
    A, U = O.operator_LU(O.case_g(c), c.labels, 25.0)
    rng = np.random.default_rng(0)
    p = np.zeros(c.labels.size)
    p[U] = rng.standard_normal(U.size)
    p = p.reshape(shape)
    ref = A @ p.ravel()[U]
    q64 = host(rw.apply_operator(vol, lab, dev(p), 25.0, "fp64", lo=lo, hi=hi)).ravel()[U]
    assert np.max(np.abs(q64 - ref)) <= 1e-12 * np.max(np.abs(ref))
    q32 = host(rw.apply_operator(vol, lab, dev(p.astype(np.float32)), 25.0, "mixed", lo=lo,
                                 hi=hi)).ravel()[U]
    assert np.max(np.abs(q32 - ref)) <= 2e-5 * np.max(np.abs(ref))


# ---------------------------------------------------------------- solves

def _oracle_same(c, tol=1e-6):
    from oracle import c_oracle
    g = O.case_g(c)
    return c_oracle.random_walker(g, c.labels, c.K, c.beta, tol=tol, return_info=True)


@pytest.fixture(scope="module")
def sphere64():
    c = sphere_case()
    ref, info = _oracle_same(c)
    return c, ref, info


def test_sphere64_fp64_parity(rw, sphere64):
    c, ref, info = sphere64
    vol, lab = _case_tensors(c)
    prob, am, st = rw.solve(vol, lab, c.K, c.beta, tol=1e-6, precision="fp64",
                            return_stats=True)
    err, ties = assert_parity(host(prob), ref, what="sphere64 fp64")
    assert st["status"] == 0
    # the fg label (2) is the solved one: same iteration count as the oracle +-1
    assert abs(st["iters"][0] - info[1]["iters"]) <= 1, (st["iters"], info)
    assert st["rel_residual"][0] <= 1.01e-6
    assert np.all(host(am) == O.argmax_labels(host(prob)))


def test_sphere64_mixed_parity(rw, sphere64):
    c, ref, info = sphere64
    vol, lab = _case_tensors(c)
    prob, am, st = rw.solve(vol, lab, c.K, c.beta, tol=1e-6, precision="mixed",
                            return_stats=True)
    assert prob.dtype.itemsize == 4
    assert_parity(host(prob), ref, what="sphere64 mixed")
    assert st["status"] == 0 and st["rel_residual"][0] <= 1e-6


@pytest.mark.parametrize("precision,mode", [("fp64", "reliable"), ("mixed", "reliable"),
                                            ("mixed", "restart")])
def test_blob_ragged_three_labels(rw, precision, mode):
    c = blob_case(shape=(37, 45, 93), n_blobs=6, K=3, seeds_per_label=40, sigma=0.08,
                  rmin=4, rmax=14, seed=11)
    ref, info = _oracle_same(c)
    vol, lab = _case_tensors(c)
    prob, am, st = rw.solve(vol, lab, c.K, c.beta, tol=1e-6, precision=precision,
                            return_stats=True, refine_mode=mode)
    assert max(st["rel_residual"]) <= 1.01e-6
    assert_parity(host(prob), ref, what=f"blob {precision}")
    seeded = c.labels > 0
    P = host(prob)
    for s in range(1, 4):
        assert np.all(P[s - 1][seeded] == (c.labels[seeded] == s))


def test_u16_volume_and_solve_all_labels(rw):
    c = blob_case(shape=(24, 40, 66), n_blobs=5, K=4, seeds_per_label=25, sigma=0.06,
                  rmin=4, rmax=12, seed=12, dtype="u16")
    ref, _ = _oracle_same(c)
    vol, lab = _case_tensors(c)
    prob, _ = rw.solve(vol, lab, c.K, c.beta, tol=1e-6, precision="fp64", solve_all_labels=True)
    P = host(prob)
    assert_parity(P, ref, what="u16 all labels")
    assert np.max(np.abs(P.sum(0) - 1)) < 1e-4


@pytest.mark.parametrize("vx,by,zc,xcd,shape", [(1, 4, 4, 0, (29, 70, 131)),
                                                (2, 4, 16, 1, (29, 70, 131)),
                                                (4, 4, 64, 1, (29, 70, 131)),
                                                (4, 4, 5, 1, (29, 70, 131)),
                                                (2, 4, 5, 0, (29, 70, 131)),
                                                (4, 4, 8, 0, (20, 33, 45)),
                                                (2, 4, 4, 1, (9, 5, 300)),
                                                (2, 8, 64, 0, (29, 70, 131)),
                                                (2, 8, 5, 1, (29, 70, 131)),
                                                (2, 8, 16, 0, (20, 33, 45)),
                                                (2, 8, 4, 1, (9, 5, 300))])
def test_tile_shapes_agree(rw, monkeypatch, vx, by, zc, xcd, shape):
    """Every tile shape (columns per lane, rows per tile, planes per tile,
    tile order; tiles wider and taller than the volume and ragged in x, y and
    z) gives the oracle's solution; float64 solves take vx = 4 as 2.  The
    9 x 5 x 300 rod is badly conditioned: stopped at relative residual 1e-6
    the oracle itself is 4e-3 from its own tol-1e-12 solution, so both sides
    solve to tight tolerances (oracle 1e-11, float64 1e-10, mixed 1e-9)."""
    c = blob_case(shape=shape, n_blobs=5, K=3, seeds_per_label=30, sigma=0.08,
                  rmin=4, rmax=12, seed=13)
    ref, _ = _oracle_same(c, tol=1e-11)
    vol, lab = _case_tensors(c)
    monkeypatch.setenv("RW_TILE_VX", str(vx))
    monkeypatch.setenv("RW_TILE_BY", str(by))
    monkeypatch.setenv("RW_TILE_ZC", str(zc))
    monkeypatch.setenv("RW_TILE_XCD", str(xcd))
    for precision, tol in (("fp64", 1e-10), ("mixed", 1e-9)):
        prob, _, st = rw.solve(vol, lab, 3, c.beta, tol=tol, precision=precision,
                               return_stats=True)
        assert st["status"] == 0
        assert st["tile"]["vx"] == (min(vx, 2) if precision == "fp64" else vx)
        assert st["tile"]["by"] == by
        assert st["tile"]["xcd"] == xcd
        assert_parity(host(prob), ref, what=f"tile vx {vx} by {by} zc {zc} {precision}")


@pytest.mark.parametrize("zc, zc2, shape", [(64, 32, (29, 70, 131)), (16, 5, (20, 33, 45)),
                                          (8, 64, (9, 5, 300))])
def test_pass2_on_its_own_tiles(rw, monkeypatch, zc, zc2, shape):
    """Mixed precision runs pass 2 on 128 x 4 x zc2 tiles beside pass 1's
    128 x 8 x zc (the 512^3 default): the oracle's solution, and within the
    stopping rule's gap of the same solve on pass 1's tiles (the partial sums
    of r.z and r.r are grouped by other tiles)."""
    c = blob_case(shape=shape, n_blobs=5, K=3, seeds_per_label=30, sigma=0.08,
                  rmin=4, rmax=12, seed=13)
    ref, _ = _oracle_same(c, tol=1e-11)
    vol, lab = _case_tensors(c)
    for k, v in (("RW_TILE_VX", 2), ("RW_TILE_BY", 8), ("RW_TILE_ZC", zc), ("RW_TILE_XCD", 0)):
        monkeypatch.setenv(k, str(v))
    same, _, st1 = rw.solve(vol, lab, 3, c.beta, tol=1e-9, precision="mixed", return_stats=True)
    assert st1["tile"]["by2"] == 8
    monkeypatch.setenv("RW_TILE_BY2", "4")
    monkeypatch.setenv("RW_TILE_ZC2", str(zc2))
    prob, _, st = rw.solve(vol, lab, 3, c.beta, tol=1e-9, precision="mixed", return_stats=True)
    assert st["status"] == 0 and st["tile"]["by"] == 8 and st["tile"]["by2"] == 4
    assert st["tile"]["zc2"] <= max(zc2, 4)
    assert_parity(host(prob), ref, what=f"pass 2 on 128 x 4 x {zc2}")
    assert np.max(np.abs(host(prob) - host(same))) <= 1e-6
    # float64 keeps one tile shape for both passes
    _, _, s64 = rw.solve(vol, lab, 3, c.beta, tol=1e-9, precision="fp64", return_stats=True)
    assert s64["tile"]["by2"] == s64["tile"]["by"]


def test_graph_and_plain_launches_bitwise_equal(rw):
    c = random_case((21, 30, 65), K=3, seeds_per_label=30, beta=40.0, seed=2)
    vol, lab = _case_tensors(c)
    a, _ = rw.solve(vol, lab, 3, 40.0, precision="fp64", use_graph=True)
    b, _ = rw.solve(vol, lab, 3, 40.0, precision="fp64", use_graph=False)
    t, _ = rw.solve(vol, lab, 3, 40.0, precision="fp64", kernel_timing=True)
    d, _ = rw.solve(vol, lab, 3, 40.0, precision="fp64", use_graph=True, check_interval=4)
    assert np.array_equal(host(a), host(b))
    assert np.array_equal(host(a), host(t))
    assert np.array_equal(host(a), host(d))


def test_warm_start_from_solution_needs_no_iterations(rw):
    c = random_case((16, 20, 24), K=2, seeds_per_label=15, beta=30.0, seed=8)
    ref, _ = _oracle_same(c, tol=1e-12)
    vol, lab = _case_tensors(c)
    x0 = dev(ref[1:2])
    prob, _, st = rw.solve(vol, lab, 2, 30.0, tol=1e-6, x0=x0, return_stats=True)
    assert st["iters"][0] == 0
    assert np.max(np.abs(host(prob) - ref)) < 1e-9


# ---------------------------------------------------------------- edge cases

@pytest.mark.parametrize("shape", [(1, 1, 7), (2, 3, 4), (1, 9, 1), (5, 1, 130)])
def test_tiny_and_degenerate_shapes(rw, shape):
    c = random_case(shape, K=2, seeds_per_label=1, beta=5.0, seed=4)
    ref = O.random_walker(O.case_g(c), c.labels, 2, 5.0, method="pcg", tol=1e-6)
    vol, lab = _case_tensors(c)
    prob, _ = rw.solve(vol, lab, 2, 5.0, tol=1e-6)
    assert_parity(host(prob), ref, what=f"shape {shape}")


def test_single_label_is_one(rw):
    c = random_case((6, 7, 8), K=1, seeds_per_label=3, beta=5.0, seed=1)
    vol, lab = _case_tensors(c)
    prob, am = rw.solve(vol, lab, 1, 5.0)
    assert np.all(host(prob) == 1.0) and np.all(host(am) == 1)


def test_constant_image(rw):
    n = 17
    vol = np.full((3, 4, n), 0.5, dtype=np.float32)
    lab = np.zeros(vol.shape, dtype=np.uint8)
    lab[:, :, 0] = 2
    lab[:, :, -1] = 1
    prob, _ = rw.solve(dev(vol), dev(lab), 2, 100.0, tol=1e-12)
    ramp = 1.0 - np.arange(n) / (n - 1)
    assert np.max(np.abs(host(prob)[1] - ramp)) < 1e-9


def test_error_statuses(rw):
    c = random_case((6, 6, 6), K=2, seeds_per_label=3, beta=5.0, seed=3)
    vol, lab = _case_tensors(c)
    with pytest.raises(rw.RWError) as e:
        rw.solve(vol, dev(np.zeros_like(c.labels)), 2, 5.0)
    assert e.value.status == rw.RW_ERR_NO_SEEDS
    lab2 = c.labels.copy()
    lab2[lab2 == 2] = 0
    with pytest.raises(rw.RWError) as e:
        rw.solve(vol, dev(lab2), 2, 5.0)
    assert e.value.status == rw.RW_ERR_NO_SEEDS
    lab3 = c.labels.copy()
    lab3[0, 0, 0] = 5
    with pytest.raises(rw.RWError) as e:
        rw.solve(vol, dev(lab3), 2, 5.0)
    assert e.value.status == rw.RW_ERR_INVALID_ARG
    with pytest.raises(rw.RWError) as e:
        rw.solve(vol, lab, 2, -1.0)
    assert e.value.status == rw.RW_ERR_INVALID_ARG
    with pytest.raises(rw.RWError) as e:
        rw.solve(vol, lab, 2, 5.0, tol=0.0)
    assert e.value.status == rw.RW_ERR_INVALID_ARG
    # singular: an unseeded voxel whose six float64 weights underflow to 0
    gs = np.zeros((3, 3, 3), dtype=np.float32)
    gs[1, 1, 1] = 1.0
    ls = np.ones((3, 3, 3), dtype=np.uint8)
    ls[1, 1, 1] = 0
    ls[0, 0, 0] = 2
    with pytest.raises(rw.RWError) as e:
        rw.solve(dev(gs), dev(ls), 2, 1000.0, precision="fp64")
    assert e.value.status == rw.RW_ERR_SINGULAR
    # non-finite input
    vn = c.vol.copy()
    vn[2, 2, 2] = np.nan
    with pytest.raises(rw.RWError) as e:
        rw.solve(dev(vn), lab, 2, 5.0, lo=0.0, hi=1.0)
    assert e.value.status == rw.RW_ERR_NONFINITE


def test_not_converged_returns_last_iterate(rw):
    c = random_case((10, 10, 10), K=2, seeds_per_label=3, beta=5.0, seed=3)
    vol, lab = _case_tensors(c)
    with pytest.warns(RuntimeWarning):
        prob, _, st = rw.solve(vol, lab, 2, 5.0, tol=1e-10, max_iter=3, return_stats=True)
    assert st["status"] == rw.RW_NOT_CONVERGED and st["iters"][0] == 3
    g = O.case_g(c)
    from oracle import c_oracle
    x, it, status, _ = c_oracle.solve_box(g, c.labels, 2, 5.0, tol=1e-10, max_iter=3)
    assert status == 1 and it == 3
    assert np.max(np.abs(host(prob)[1] - x)) < 1e-12


def test_workspace_too_small(rw):
    import ctypes
    import torch
    c = random_case((6, 6, 6), K=2, seeds_per_label=3, beta=5.0, seed=3)
    vol, lab = _case_tensors(c)
    # the binding allocates a fresh workspace when the given one is too small,
    # so call the ABI directly with a short one
    V = rw.make_volume(vol)
    S = rw._seeds(lab, 2)
    o = rw.options(5.0)
    prob = torch.empty((2, 6, 6, 6), dtype=torch.float64, device="cuda")
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    st = rw.lib().rw_solve(rw.default_context().handle, ctypes.byref(V), ctypes.byref(S),
                           ctypes.byref(o), rw._ptr(prob), None, rw._ptr(ws), 16, None,
                           rw._stream())
    assert st == rw.RW_ERR_WORKSPACE


def test_autotuner_records_a_tile_and_solves_agree(rw):
    c = blob_case(shape=(48, 64, 96), n_blobs=5, K=3, seeds_per_label=30, sigma=0.08,
                  rmin=4, rmax=12, seed=17)
    vol, lab = _case_tensors(c)
    ref, _ = _oracle_same(c)
    vx, zc, xcd, by = rw.autotune(vol, lab, 3, c.beta, precision="mixed")
    assert vx in (1, 2, 4) and zc in (16, 32, 64) and xcd in (0, 1) and by in (4, 8)
    assert by == 4 or vx == 2
    prob, _, st = rw.solve(vol, lab, 3, c.beta, precision="mixed", return_stats=True)
    assert st["tile"]["vx"] == vx and st["tile"]["xcd"] == xcd and st["tile"]["by"] == by
    assert_parity(host(prob), ref, what="after autotune")


def test_tile_table_file_is_written_and_read_by_later_processes(tmp_path):
    """The autotuner's table outlives its process: a child process tunes a
    volume (RW_TUNE_FILE = a fresh file) and the file then names the shape;
    a second child process solves the same volume and reports the tuned shape
    as coming from the table; with RW_TUNE_FILE empty the built-in shape is
    used."""
    import json
    import subprocess
    import sys
    import textwrap
    path = tmp_path / "librw.tune"
    code = textwrap.dedent("""
        import json, sys
        import numpy as np
        sys.path.insert(0, %r)
        from synth import blob_case
        from paper_2509_26213_amd import rw
        from tests._helpers import dev
        c = blob_case(shape=(40, 60, 200), n_blobs=6, K=3, seeds_per_label=30, sigma=0.06,
                      rmin=5, rmax=12, seed=91)
        vol, lab = dev(c.vol), dev(c.labels)
        best = rw.autotune(vol, lab, 3, c.beta, precision="mixed") if sys.argv[1] == "tune" else None
        _, _, st = rw.solve(vol, lab, 3, c.beta, precision="mixed", return_stats=True)
        print(json.dumps(dict(best=best, tile=st["tile"], tuned=st["tile_tuned"])))
    """ % ROOT_DIR)
    env = dict(os.environ, RW_TUNE_FILE=str(path))
    first = subprocess.run([sys.executable, "-c", code, "tune"], env=env, capture_output=True,
                           text=True, timeout=600)
    assert first.returncode == 0, first.stderr[-2000:]
    r1 = json.loads(first.stdout.strip().splitlines()[-1])
    assert path.exists() and "whole 1 2 " in path.read_text()
    second = subprocess.run([sys.executable, "-c", code, "solve"], env=env, capture_output=True,
                            text=True, timeout=600)
    assert second.returncode == 0, second.stderr[-2000:]
    r2 = json.loads(second.stdout.strip().splitlines()[-1])
    vx, zc, xcd, by = r1["best"]
    t2 = r2["tile"]
    assert r2["tuned"] and (t2["vx"], t2["by"], t2["xcd"]) == (vx, by, xcd)
    off = subprocess.run([sys.executable, "-c", code, "solve"],
                         env=dict(os.environ, RW_TUNE_FILE=""), capture_output=True, text=True,
                         timeout=600)
    assert off.returncode == 0, off.stderr[-2000:]
    assert not json.loads(off.stdout.strip().splitlines()[-1])["tuned"]
