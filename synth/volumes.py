"""Seeded synthetic volumes and seed maps.

Conventions (all arrays C order ``[nz][ny][nx]``, x fastest):

* ``labels`` is a uint8 map: 0 = unseeded, 1..K = seed label, label 1 is the
  background class.
* ``truth`` is the generator's own class map (1..K) or, for the sphere cases,
  a boolean foreground mask.  It is ground truth for seed sampling and for the
  differentiable-loss case; the solver never sees it.
* Every random draw comes from ``numpy.random.default_rng(seed)`` in a fixed
  order: blob parameters, then the volume noise (z-slab by z-slab), then the
  seeds label by label in label order.  The brick-wise generator instead uses a
  counter-based hash (SplitMix64) of the global voxel index, so any brick can
  be produced on its own, in any order, with identical values.

Nothing here computes edge weights, Laplacians or solves.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Case:
    name: str
    vol: np.ndarray            # float32 or uint16, [nz][ny][nx]
    labels: np.ndarray         # uint8, [nz][ny][nx]
    K: int                     # number of labels
    beta: float
    norm: str                  # "minmax" (float32 input) or "u16" (divide by 65535)
    truth: Optional[np.ndarray] = None
    params: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.vol.shape

    def norm_range(self):
        """(lo, hi) of the affine normalisation g = (v - lo) / (hi - lo)."""
        if self.norm == "u16":
            return 0.0, 65535.0
        return float(self.vol.min()), float(self.vol.max())


# --------------------------------------------------------------------------
# seed sampling
# --------------------------------------------------------------------------

def _sample_region(rng, region_fn, n_total, count, taken, batch=None):
    """Draw ``count`` distinct flat indices whose region test is true.

    Rejection sampling with uniform draws over the whole grid; duplicates and
    already-taken voxels are discarded, so the sample is without replacement.
    ``region_fn(flat_idx) -> bool array``.
    """
    out = []
    seen = set()
    batch = batch or max(4 * count, 1024)
    while len(out) < count:
        cand = rng.integers(0, n_total, size=batch, dtype=np.int64)
        ok = region_fn(cand)
        for c in cand[ok]:
            c = int(c)
            if c in seen or c in taken:
                continue
            seen.add(c)
            out.append(c)
            if len(out) == count:
                break
    return np.asarray(out, dtype=np.int64)


def _paint_seeds(rng, shape, K, per_label, region_of_label):
    n_total = int(np.prod(shape))
    labels = np.zeros(n_total, dtype=np.uint8)
    taken = set()
    for s in range(1, K + 1):
        cnt = per_label[s - 1] if isinstance(per_label, (list, tuple)) else per_label
        idx = _sample_region(rng, region_of_label(s), n_total, cnt, taken)
        labels[idx] = s
        taken.update(int(i) for i in idx)
    return labels.reshape(shape)


def _unravel(flat, shape):
    nz, ny, nx = shape
    z = flat // (ny * nx)
    rem = flat - z * (ny * nx)
    y = rem // nx
    x = rem - y * nx
    return z, y, x


# --------------------------------------------------------------------------
# sphere cases (small plain solve, differentiable case)
# --------------------------------------------------------------------------

def sphere_case(n=64, radius=20.0, fg=0.7, bg=0.3, sigma=0.05, seed_radius=10.0,
                corner=8, n_seeds=200, beta=100.0, seed=1, name="sphere64"):
    """Centered sphere on a flat background with Gaussian noise, two labels.

    Label 1 (background) seeds lie in the eight corner ``corner^3`` cubes,
    label 2 (foreground) seeds within ``seed_radius`` of the centre.  The
    centre is ((n-1)/2,)*3 and "inside" includes the boundary.
    """
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    c = (n - 1) / 2.0
    z, y, x = np.ogrid[:n, :n, :n]
    d2 = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2
    inside = d2 <= radius * radius
    base = np.where(inside, fg, bg).astype(np.float64)
    vol = (base + rng.normal(0.0, sigma, size=shape)).astype(np.float32)

    def region(s):
        def fn(flat):
            zz, yy, xx = _unravel(flat, shape)
            if s == 1:
                def lo_hi(a):
                    return (a < corner) | (a >= n - corner)
                return lo_hi(zz) & lo_hi(yy) & lo_hi(xx)
            dd = (xx - c) ** 2 + (yy - c) ** 2 + (zz - c) ** 2
            return dd <= seed_radius * seed_radius
        return fn

    labels = _paint_seeds(rng, shape, 2, n_seeds, region)
    return Case(name=name, vol=vol, labels=labels, K=2, beta=beta, norm="minmax",
                truth=inside, params=dict(n=n, radius=radius, sigma=sigma, seed=seed))


# --------------------------------------------------------------------------
# blob cases (multi-label solve, hierarchy)
# --------------------------------------------------------------------------

def _blob_params(rng, shape, n_blobs, rmin, rmax, K):
    nz, ny, nx = shape
    centres = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * np.array([nz, ny, nx], dtype=np.float64)
    radii = rng.uniform(rmin, rmax, size=(n_blobs, 3))
    inten = rng.uniform(0.5, 0.9, size=n_blobs)
    cls = np.array([2 + (i % (K - 1)) for i in range(n_blobs)], dtype=np.uint8)
    return centres, radii, inten, cls


def _paint_blobs(base, cmap, z0, centres, radii, inten, cls):
    """Paint axis-aligned ellipsoids (painter's order) into a z-slab starting at z0."""
    sz, ny, nx = base.shape
    for (cz, cy, cx), (rz, ry, rx), v, k in zip(centres, radii, inten, cls):
        zlo, zhi = max(int(np.floor(cz - rz)), z0), min(int(np.ceil(cz + rz)) + 1, z0 + sz)
        ylo, yhi = max(int(np.floor(cy - ry)), 0), min(int(np.ceil(cy + ry)) + 1, ny)
        xlo, xhi = max(int(np.floor(cx - rx)), 0), min(int(np.ceil(cx + rx)) + 1, nx)
        if zlo >= zhi or ylo >= yhi or xlo >= xhi:
            continue
        zz = (np.arange(zlo, zhi, dtype=np.float64)[:, None, None] - cz) / rz
        yy = (np.arange(ylo, yhi, dtype=np.float64)[None, :, None] - cy) / ry
        xx = (np.arange(xlo, xhi, dtype=np.float64)[None, None, :] - cx) / rx
        m = (zz * zz + yy * yy + xx * xx) <= 1.0
        sub_b = base[zlo - z0:zhi - z0, ylo:yhi, xlo:xhi]
        sub_c = cmap[zlo - z0:zhi - z0, ylo:yhi, xlo:xhi]
        sub_b[m] = v
        sub_c[m] = k


def _class_at(points_zyx, centres, radii, cls):
    """Class (1 = background) of integer voxel positions under painter's order."""
    z, y, x = (np.asarray(a, dtype=np.float64) for a in points_zyx)
    out = np.ones(z.shape, dtype=np.uint8)
    for (cz, cy, cx), (rz, ry, rx), k in zip(centres, radii, cls):
        m = ((z - cz) / rz) ** 2 + ((y - cy) / ry) ** 2 + ((x - cx) / rx) ** 2 <= 1.0
        out[m] = k
    return out


def blob_case(shape=(512, 512, 512), n_blobs=32, K=3, seeds_per_label=1000, sigma=0.08,
              bg=0.2, rmin=10.0, rmax=60.0, beta=150.0, seed=2, dtype="f32",
              name=None, slab=64):
    """Ellipsoid "cells" on a background, K-1 blob classes plus background.

    Blob i has class 2 + (i mod (K-1)); later blobs paint over earlier ones.
    Noise N(0, sigma^2) is added in float64 and the sum is cast to float32
    (``dtype="f32"``) or stored as round(clip(v, 0, 1) * 65535) (``"u16"``).
    """
    if isinstance(shape, int):
        shape = (shape, shape, shape)
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    centres, radii, inten, cls = _blob_params(rng, shape, n_blobs, rmin, rmax, K)
    nz, ny, nx = shape
    out = np.empty(shape, dtype=np.float32 if dtype == "f32" else np.uint16)
    truth = np.empty(shape, dtype=np.uint8)
    for z0 in range(0, nz, slab):
        sz = min(slab, nz - z0)
        base = np.full((sz, ny, nx), bg, dtype=np.float64)
        cmap = np.ones((sz, ny, nx), dtype=np.uint8)
        _paint_blobs(base, cmap, z0, centres, radii, inten, cls)
        base += rng.normal(0.0, sigma, size=base.shape)
        if dtype == "f32":
            out[z0:z0 + sz] = base.astype(np.float32)
        else:
            out[z0:z0 + sz] = np.rint(np.clip(base, 0.0, 1.0) * 65535.0).astype(np.uint16)
        truth[z0:z0 + sz] = cmap

    flat_truth = truth.reshape(-1)

    def region(s):
        return lambda flat: flat_truth[flat] == s

    labels = _paint_seeds(rng, shape, K, seeds_per_label, region)
    return Case(name=name or f"blob{nz}x{ny}x{nx}", vol=out, labels=labels, K=K, beta=beta,
                norm="minmax" if dtype == "f32" else "u16", truth=truth,
                params=dict(shape=shape, n_blobs=n_blobs, seeds_per_label=seeds_per_label,
                            sigma=sigma, rmin=rmin, rmax=rmax, seed=seed, dtype=dtype))


def random_case(shape=(8, 8, 8), K=2, seeds_per_label=4, beta=10.0, seed=0, dtype="f32"):
    """Uniform random intensities in [0,1) with random seeds (tiny pin cases)."""
    if isinstance(shape, int):
        shape = (shape, shape, shape)
    rng = np.random.default_rng(seed)
    vol = rng.random(shape).astype(np.float32)
    if dtype == "u16":
        vol = np.rint(vol * 65535.0).astype(np.uint16)
    n_total = int(np.prod(shape))
    perm = rng.permutation(n_total)
    labels = np.zeros(n_total, dtype=np.uint8)
    k = 0
    for s in range(1, K + 1):
        cnt = seeds_per_label[s - 1] if isinstance(seeds_per_label, (list, tuple)) else seeds_per_label
        labels[perm[k:k + cnt]] = s
        k += cnt
    return Case(name=f"random{shape}", vol=vol, labels=labels.reshape(shape), K=K, beta=beta,
                norm="minmax" if dtype == "f32" else "u16",
                params=dict(shape=shape, seed=seed))


# --------------------------------------------------------------------------
# brick-wise generator (counter-based, order independent)
# --------------------------------------------------------------------------

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x):
    """SplitMix64 finaliser (Steele, Lea, Flood 2014) on a uint64 array."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _hash_normal(seed, flat_idx):
    """N(0,1) sample per global index: two SplitMix64 uniforms, Box-Muller."""
    flat_idx = np.asarray(flat_idx, dtype=np.uint64)
    key = splitmix64(np.uint64(seed))
    with np.errstate(over="ignore"):
        a = splitmix64(key ^ (flat_idx * np.uint64(2)))
        b = splitmix64(key ^ (flat_idx * np.uint64(2) + np.uint64(1)))
    # 53-bit uniforms in (0, 1]
    u1 = ((a >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)
    u2 = (b >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


class brickwise_blob_case:
    """A large u16 blob volume that is never materialised whole.

    ``brick(origin, size)`` returns the u16 values and seed labels of any box
    (with no halo logic: ask for the halo explicitly).  Blob parameters and
    seed positions come from ``default_rng(seed)``; the noise of voxel k is
    ``_hash_normal(seed, k)``.
    """

    def __init__(self, shape=(1024, 2048, 2048), n_blobs=1024, K=4, seeds_per_label=4000,
                 sigma=0.08, bg=0.2, rmin=10.0, rmax=60.0, beta=150.0, seed=5):
        self.shape = tuple(int(s) for s in shape)
        self.K, self.beta, self.sigma, self.bg, self.seed = K, beta, sigma, bg, seed
        self.norm = "u16"
        rng = np.random.default_rng(seed)
        self.centres, self.radii, self.inten, self.cls = _blob_params(
            rng, self.shape, n_blobs, rmin, rmax, K)
        n_total = int(np.prod(self.shape))

        def region(s):
            def fn(flat):
                return _class_at(_unravel(flat, self.shape), self.centres, self.radii, self.cls) == s
            return fn

        seeds = []
        taken = set()
        for s in range(1, K + 1):
            idx = _sample_region(rng, region(s), n_total, seeds_per_label, taken)
            taken.update(int(i) for i in idx)
            seeds.append(idx)
        self.seed_idx = np.concatenate(seeds)
        self.seed_lab = np.concatenate([np.full(len(a), s + 1, np.uint8) for s, a in enumerate(seeds)])
        order = np.argsort(self.seed_idx)
        self.seed_idx, self.seed_lab = self.seed_idx[order], self.seed_lab[order]

    def brick(self, origin, size):
        oz, oy, ox = (int(v) for v in origin)
        sz, sy, sx = (int(v) for v in size)
        nz, ny, nx = self.shape
        base = np.full((sz, sy, sx), self.bg, dtype=np.float64)
        cmap = np.ones((sz, sy, sx), dtype=np.uint8)
        # paint in local coordinates by shifting the centres
        cen = self.centres - np.array([0.0, oy, ox])
        sub = np.zeros((sz, sy, sx), dtype=np.float64)
        sub[:] = base
        _paint_blobs(sub, cmap, oz, cen, self.radii, self.inten, self.cls)
        zz, yy, xx = np.meshgrid(np.arange(oz, oz + sz, dtype=np.uint64),
                                 np.arange(oy, oy + sy, dtype=np.uint64),
                                 np.arange(ox, ox + sx, dtype=np.uint64), indexing="ij")
        flat = (zz * np.uint64(ny) + yy) * np.uint64(nx) + xx
        sub += self.sigma * _hash_normal(self.seed, flat)
        vol = np.rint(np.clip(sub, 0.0, 1.0) * 65535.0).astype(np.uint16)
        labels = np.zeros((sz, sy, sx), dtype=np.uint8)
        lo = np.searchsorted(self.seed_idx, 0)
        z, y, x = _unravel(self.seed_idx[lo:], self.shape)
        inb = (z >= oz) & (z < oz + sz) & (y >= oy) & (y < oy + sy) & (x >= ox) & (x < ox + sx)
        labels[z[inb] - oz, y[inb] - oy, x[inb] - ox] = self.seed_lab[lo:][inb]
        return vol, labels, cmap


# --------------------------------------------------------------------------
# volume time series (4-D random walker)
# --------------------------------------------------------------------------

def timeseries_case(shape=(200, 50, 224, 224), radius=(14.0, 40.0, 40.0), amplitude=0.25,
                    fg=0.7, bg=0.3, sigma=0.05, fg_seeds_first=10, bg_seeds_first=10,
                    fg_seeds_last=4, beta=100.0, seed=6, name="heart4d"):
    """A volume time series [nt][nz][ny][nx] standing in for a cardiac MRI
    sequence: an ellipsoid at the centre of every time step whose radii
    (rz, ry, rx) pulse as r (1 + amplitude sin(2 pi t / nt)), intensity fg on
    bg, additive Gaussian noise sigma.  Two labels: label 2 (foreground) seeds
    inside the ellipsoid at half its radii, label 1 (background) seeds outside
    1.5 times its radii; fg_seeds_first and bg_seeds_first seeds in time step
    0, fg_seeds_last foreground seeds in the last time step.  float32."""
    rng = np.random.default_rng(seed)
    nt, nz, ny, nx = shape
    cz, cy, cx = (nz - 1) / 2.0, (ny - 1) / 2.0, (nx - 1) / 2.0
    z, y, x = np.ogrid[:nz, :ny, :nx]
    vol = np.empty(shape, np.float32)
    truth = np.empty(shape, bool)
    scale = 1.0 + amplitude * np.sin(2.0 * np.pi * np.arange(nt) / nt)
    for t in range(nt):
        rz, ry, rx = (r * scale[t] for r in radius)
        inside = ((z - cz) / rz) ** 2 + ((y - cy) / ry) ** 2 + ((x - cx) / rx) ** 2 <= 1.0
        truth[t] = inside
        vol[t] = (np.where(inside, fg, bg) + rng.normal(0.0, sigma, size=(nz, ny, nx))).astype(
            np.float32)
    labels = np.zeros(shape, np.uint8)
    n3 = nz * ny * nx

    def draw(t, count, lab, lo, hi):
        rz, ry, rx = (r * scale[t] for r in radius)
        got = 0
        while got < count:
            f = int(rng.integers(0, n3))
            zz, yy, xx = _unravel(np.int64(f), (nz, ny, nx))
            e = ((zz - cz) / rz) ** 2 + ((yy - cy) / ry) ** 2 + ((xx - cx) / rx) ** 2
            if lo <= e <= hi and labels[t, zz, yy, xx] == 0:
                labels[t, zz, yy, xx] = lab
                got += 1

    draw(0, fg_seeds_first, 2, 0.0, 0.25)
    draw(0, bg_seeds_first, 1, 2.25, np.inf)
    draw(nt - 1, fg_seeds_last, 2, 0.0, 0.25)
    return Case(name=name, vol=vol, labels=labels, K=2, beta=beta, norm="minmax", truth=truth,
                params=dict(shape=shape, radius=radius, amplitude=amplitude, sigma=sigma,
                            seed=seed))
