"""Pins of the oracle's 4-D random walker (a volume time series [nt][nz][ny][nx]
as one 8-connected grid: the two neighbours along x, y, z and t), the form
the paper applies to a cardiac MRI time series (Sec. V-B)."""
import numpy as np
import pytest

from oracle import rw_oracle as O
from synth import timeseries_case


def test_edge_set_is_eight_connected():
    shape = (3, 4, 5, 6)
    i, j, a = O.grid_edges(shape)
    nt, nz, ny, nx = shape
    assert i.size == (nt * nz * ny * (nx - 1) + nt * nz * (ny - 1) * nx
                      + nt * (nz - 1) * ny * nx + (nt - 1) * nz * ny * nx)
    deg = np.bincount(np.r_[i, j], minlength=int(np.prod(shape))).reshape(shape)
    assert deg[1, 1, 1, 1] == 8 and deg[0, 0, 0, 0] == 4
    # a t edge joins the same voxel of consecutive time steps
    step = nz * ny * nx
    assert np.all((j - i)[a == 3] == step)
    assert np.all((j - i)[a == 2] == ny * nx)


def test_ramp_along_time_on_a_constant_image():
    """Constant image, fg in the whole first time step, bg in the last: the
    harmonic function is linear in t, x_fg = 1 - t / (nt - 1)."""
    shape = (7, 3, 4, 5)
    g = np.full(shape, 0.4)
    lab = np.zeros(shape, np.uint8)
    lab[0] = 2
    lab[-1] = 1
    ramp = 1.0 - np.arange(7) / 6.0
    for method in ("dense", "pcg"):
        x = O.random_walker(g, lab, 2, 30.0, method=method, tol=1e-13)[1]
        assert np.max(np.abs(x - ramp[:, None, None, None])) < 1e-11


def test_resistor_divider_along_time():
    """Image varying only along t, seed planes at both ends: the 1-D divider
    with resistances exp(beta dg_k^2) between consecutive time steps."""
    nt, beta = 9, 25.0
    prof = np.random.default_rng(4).random(nt)
    g = np.broadcast_to(prof[:, None, None, None], (nt, 2, 3, 3)).copy()
    lab = np.zeros(g.shape, np.uint8)
    lab[0] = 2
    lab[-1] = 1
    R = np.exp(beta * np.diff(prof) ** 2)
    expect = np.array([R[k:].sum() / R.sum() for k in range(nt)])
    x = O.random_walker(g, lab, 2, beta, method="direct")[1]
    assert np.max(np.abs(x - expect[:, None, None, None])) < 1e-12


def test_time_invariant_series_equals_the_single_volume():
    """The same volume and seeds at every time step: t edges carry no current,
    so every time step holds the 3-D solution of one volume."""
    rng = np.random.default_rng(2)
    g3 = rng.random((4, 5, 6))
    lab3 = np.zeros(g3.shape, np.uint8)
    flat = rng.permutation(g3.size)
    lab3.flat[flat[:3]] = 1
    lab3.flat[flat[3:6]] = 2
    lab3.flat[flat[6:8]] = 3
    x3 = O.random_walker(g3, lab3, 3, 12.0, method="dense")
    g4 = np.broadcast_to(g3, (5,) + g3.shape).copy()
    lab4 = np.broadcast_to(lab3, (5,) + g3.shape).copy()
    x4 = O.random_walker(g4, lab4, 3, 12.0, method="direct")
    for t in range(5):
        assert np.max(np.abs(x4[:, t] - x3)) < 1e-12


@pytest.mark.parametrize("perm", [(3, 1, 2, 0), (1, 0, 3, 2)])
def test_axis_permutation_equivariance_4d(perm):
    rng = np.random.default_rng(8)
    g = rng.random((3, 4, 5, 4))
    lab = np.zeros(g.shape, np.uint8)
    flat = rng.permutation(g.size)
    lab.flat[flat[:4]] = 1
    lab.flat[flat[4:8]] = 2
    x = O.random_walker(g, lab, 2, 9.0, method="dense")
    xt = O.random_walker(np.ascontiguousarray(g.transpose(perm)),
                         np.ascontiguousarray(lab.transpose(perm)), 2, 9.0, method="dense")
    for k in range(2):
        assert np.max(np.abs(xt[k] - x[k].transpose(perm))) < 1e-12


def test_timeseries_case_pcg_invariants():
    """The synthetic time series at a small size: Jacobi-PCG agrees with the
    sparse direct solve, 0 <= x <= 1 (within the tolerance), the labels sum to
    one and seeds are exact."""
    c = timeseries_case(shape=(6, 8, 10, 12), radius=(2.5, 3.0, 4.0), fg_seeds_first=6,
                        bg_seeds_first=6, fg_seeds_last=3, seed=3)
    g = O.case_g(c)
    xe = O.random_walker(g, c.labels, 2, c.beta, method="direct")
    xp, info = O.random_walker(g, c.labels, 2, c.beta, method="pcg", tol=1e-10,
                               return_info=True)
    assert np.max(np.abs(xe - xp)) < 1e-7
    assert xe.min() >= -1e-12 and xe.max() <= 1 + 1e-12
    assert np.max(np.abs(xe.sum(0) - 1)) < 1e-12
    seeded = c.labels > 0
    assert np.all(xe[1][seeded] == (c.labels[seeded] == 2))
    # the foreground seeds of the last time step reach it through time only
    assert xe[1][-1][c.truth[-1]].mean() > 0.5
