"""GPU parity of the 4-D random walker (a volume time series [nt][nz][ny][nx]
as one 8-connected grid, Sec. V-B) against the oracle's assembled 4-D
system: the step-by-step Jacobi-PCG at tol 1e-6 on the solved labels, every
label and the argmax at tol 1e-10, both precisions; a single time step equals
the 3-D solve bit for bit; a time-invariant series solves like one volume."""
import numpy as np
import pytest

from oracle import rw_oracle as O
from synth import timeseries_case
from tests._helpers import assert_parity, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rw():
    from paper_2509_26213_amd import rw as m
    m.lib()
    return m


def _random4d(shape, K, per_label, beta, seed):
    """Random intensities in [0, 1] with a smooth component (so the weights
    vary over decades) and `per_label` random seeds per label."""
    rng = np.random.default_rng(seed)
    nt, nz, ny, nx = shape
    t, z, y, x = np.meshgrid(*(np.linspace(0, 1, n) for n in shape), indexing="ij")
    vol = 0.5 + 0.3 * np.sin(3 * x + 2 * y) * np.cos(2 * z - t) + 0.1 * rng.standard_normal(shape)
    vol = vol.astype(np.float32)
    lab = np.zeros(shape, np.uint8)
    free = rng.permutation(lab.size)[:K * per_label]
    for k in range(K):
        lab.ravel()[free[k * per_label:(k + 1) * per_label]] = k + 1
    return vol, lab, beta


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_random_series_matches_oracle(rw, precision):
    """Ragged 4-D grid (tiles straddle time steps), three labels: at tol 1e-6
    the solved labels follow the oracle's step-by-step solve (float64: the
    same iteration counts to within one); at tol 1e-10 every label and the
    argmax meet the parity bar."""
    vol, lab, beta = _random4d((5, 7, 11, 70), 3, 12, 25.0, seed=71)
    lo, hi = float(vol.min()), float(vol.max())
    g = O.normalize(vol, lo, hi)
    ref6, info6 = O.random_walker(g, lab, 3, beta, method="pcg", tol=1e-6, solve_labels=[2, 3],
                                  return_info=True)
    prob, _, st = rw.solve4d(dev(vol), dev(lab), 3, beta, tol=1e-6, precision=precision,
                             return_stats=True)
    assert st["status"] == 0 and st["num_solved"] == 2
    err = np.max(np.abs(host(prob)[1:] - ref6))
    assert err <= 1e-5, err
    if precision == "fp64":
        for r in range(2):
            assert abs(st["iters"][r] - info6[r]["iters"]) <= 1, (st["iters"], info6)
    ref = O.random_walker(g, lab, 3, beta, method="direct")
    prob, am, st = rw.solve4d(dev(vol), dev(lab), 3, beta, tol=1e-10, precision=precision,
                              return_stats=True)
    assert st["status"] == 0
    P = host(prob)
    assert_parity(P, ref, what=f"4-D {precision}")
    assert np.array_equal(host(am), (np.argmax(P, axis=0) + 1).astype(np.uint8))
    seeded = lab > 0
    for s in (1, 2, 3):
        assert np.all(P[s - 1][seeded] == (lab[seeded] == s))


@pytest.fixture(scope="module")
def ellipsoid4d():
    """The synthetic cardiac stand-in at a small size (12 time steps of
    10 x 24 x 24, seeds in the first and last time step only, as in the
    paper's experiment) and the oracle's float64 Jacobi-PCG solve of both
    labels at tol 1e-12 (a direct factorisation of this 4-D Laplacian fills
    in far more than a 3-D one and takes minutes)."""
    c = timeseries_case(shape=(12, 10, 24, 24), radius=(3.0, 7.0, 7.0), fg_seeds_first=10,
                        bg_seeds_first=10, fg_seeds_last=4, seed=6)
    ref = O.random_walker(O.case_g(c), c.labels, 2, c.beta, method="pcg", tol=1e-12)
    return c, ref


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pulsing_ellipsoid_series_matches_oracle(rw, ellipsoid4d, precision):
    """Every label within 1e-5 of the oracle at tol 1e-10."""
    c, ref = ellipsoid4d
    prob, am, st = rw.solve4d(dev(c.vol), dev(c.labels), 2, c.beta, tol=1e-10,
                              precision=precision, return_stats=True)
    assert st["status"] == 0
    assert_parity(host(prob), ref, what=f"pulsing ellipsoid {precision}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_single_time_step_equals_3d_solve(rw, precision):
    """nt = 1: no time edges, so the 4-D solve is the 3-D solve, bit for bit."""
    vol, lab, beta = _random4d((1, 9, 13, 70), 3, 10, 25.0, seed=72)
    p4, a4 = rw.solve4d(dev(vol), dev(lab), 3, beta, tol=1e-6, precision=precision)
    p3, a3 = rw.solve(dev(vol[0]), dev(lab[0]), 3, beta, tol=1e-6, precision=precision)
    assert np.array_equal(host(p4)[:, 0], host(p3))
    assert np.array_equal(host(a4)[0], host(a3))


def test_time_invariant_series_solves_like_one_volume(rw):
    """Every time step the same image and the same seeds: no flow along t,
    so each time step holds the 3-D solution of that volume."""
    vol, lab, beta = _random4d((1, 8, 12, 66), 2, 10, 25.0, seed=73)
    v4 = np.repeat(vol, 6, axis=0)
    l4 = np.repeat(lab, 6, axis=0)
    lo, hi = float(vol.min()), float(vol.max())
    p4, _ = rw.solve4d(dev(v4), dev(l4), 2, beta, tol=1e-11, precision="fp64", lo=lo, hi=hi)
    p3, _ = rw.solve(dev(vol[0]), dev(lab[0]), 2, beta, tol=1e-11, precision="fp64", lo=lo, hi=hi)
    P4, P3 = host(p4), host(p3)
    for t in range(6):
        assert np.max(np.abs(P4[:, t] - P3)) <= 1e-8, t


def test_bad_time_steps_are_refused(rw):
    import torch
    vol = torch.zeros((2, 3, 4, 5), dtype=torch.float32, device="cuda")
    lab = torch.zeros((2, 3, 4, 5), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        rw.solve4d(vol, lab[0], 2, 1.0)
    lab[0, 0, 0, 0], lab[1, 2, 3, 4] = 1, 2
    prob, _ = rw.solve4d(vol, lab, 2, 1.0, tol=1e-10, lo=0.0, hi=1.0)
    # constant image: x_fg is harmonic with unit weights; spot-check the seeds
    assert float(prob[1, 1, 2, 3, 4]) == 1.0 and float(prob[1, 0, 0, 0, 0]) == 0.0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_series_and_plain_tile_orders_agree(rw, precision, monkeypatch):
    """The time-series tile order (chunks within one time step, steps
    interleaved) and the plain volume order (chunks straddling steps) solve
    the same system: equal within the tol-1e-10 gap.  Here both take
    4-plane chunks: [0, 4), [4, 8), [8, 9) of every step against chunks
    that straddle each step boundary, so the partial sums differ."""
    vol, lab, beta = _random4d((6, 9, 13, 140), 3, 12, 25.0, seed=74)
    p_s, a_s, st_s = rw.solve4d(dev(vol), dev(lab), 3, beta, tol=1e-10, precision=precision,
                                return_stats=True)
    monkeypatch.setenv("RW_SERIES_PLAIN", "1")
    p_p, a_p, st_p = rw.solve4d(dev(vol), dev(lab), 3, beta, tol=1e-10, precision=precision,
                                return_stats=True)
    assert st_s["status"] == 0 and st_p["status"] == 0
    assert st_s["tile"]["zc"] == 4 and st_p["tile"]["zc"] == 4
    bound = 1e-8 if precision == "fp64" else 2e-6
    assert np.max(np.abs(host(p_s) - host(p_p))) <= bound
